"""GPU parity on Example 1 of Sec. 3 (bilinear finite elements for
anisotropic diffusion, 160 x 160 elements, 4 levels), through the C ABI's
9-point-stencil setup, against the FP64 oracle on the quadrature-assembled
matrix.

Setup of the runs (the paper's work per level, damped Jacobi for SSOR):
MPCG with m = 5 and nu = 6, additive MG-PCG with nu = 6, MG(V)-PCG with
3 + 3 sweeps; omega = 1/2 (lambda_max(D^-1 A) -> 3 as kxx -> 0).  Bars:
iterates at equal k to 1e-10 relative, converged counts within one,
alpha histories to 1e-8 of the largest |alpha| where every Gram kept full
rank, FP32 bulk true residual <= 1e-8; Sec. 3's ordering and alpha
observations on the GPU's own history.
"""
import numpy as np
import pytest

import workloads as W
from oracle import comparators as C
from oracle import fem, hierarchy, mpcg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_12833_amd as amg  # noqa: E402

M = W.EXAMPLE1_ELEMENTS
N1 = M - 1
OPTS = dict(m=5, nu=6, omega=0.5, maxit=3000)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    amg.load()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def rel(a, b):
    """max(normwise, element-wise max |a - b| / max |b|) relative error."""
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    return max(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0),
               (np.abs(a - b).max() / mb) if mb > 0 else 0.0)


def oracle_h(kxx):
    return hierarchy.build(2, N1, W.EXAMPLE1_LEVELS, A=fem.stiffness(M, kxx))


@pytest.mark.parametrize("kxx", [1.0, 1e-1, 1e-6])
def test_example1_mpcg_matches_oracle(kxx):
    h = oracle_h(kxx)
    b = fem.load(M)
    s = amg.Solver(2, N1, W.EXAMPLE1_LEVELS, stencil=W.example1_stencil(kxx), **OPTS)
    bg = dev(W.example1_rhs())
    for k in (1, 5, 20):
        o = mpcg.mpcg(h, b, tol=0.0, maxit=k, m=5, nu=6, omega=0.5)
        xg, inf = s.solve(bg, tol=0.0, maxit=k)
        assert inf["iterations"] == k
        assert rel(xg.cpu().numpy(), o.x) <= 1e-10, (kxx, k, rel(xg.cpu().numpy(), o.x))
    ref = mpcg.mpcg(h, b, tol=1e-8, m=5, nu=6, omega=0.5, maxit=3000)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and abs(info["iterations"] - ref.iterations) <= 1, (info, ref.iterations)
    rt = s.residual(bg, x)
    assert float(torch.linalg.norm(rt) / torch.linalg.norm(bg)) <= 1.01e-8
    alph, _ = s.history()
    k = min(len(alph), len(ref.alphas), 30)
    if all(r == W.EXAMPLE1_LEVELS for r in ref.ranks[:k]):
        A_o = np.array(ref.alphas[:k])
        assert np.abs(alph[:k] - A_o).max() <= 1e-8 * np.abs(A_o).max()
    s.close()


def test_example1_alpha_observations_on_the_gpu():
    """Sec. 3, high anisotropy: some alpha_l are negative; in the later
    iterations the finest level carries the largest |alpha_l| and the coarse
    ones have shrunk."""
    s = amg.Solver(2, N1, W.EXAMPLE1_LEVELS, stencil=W.example1_stencil(1e-6), **OPTS)
    _, info = s.solve(dev(W.example1_rhs()), tol=1e-8)
    assert info["status"] == amg.OK
    al, _ = s.history()
    assert (al < 0).any()
    late, early = np.abs(al[-10:]), np.abs(al[:10])
    assert (late.argmax(axis=1) == al.shape[1] - 1).all()
    assert late[:, :-1].mean() < 0.5 * early[:, :-1].mean()
    s.close()


def test_example1_comparators_and_ordering():
    kxx = 1e-6
    h = oracle_h(kxx)
    b = fem.load(M)
    st = W.example1_stencil(kxx)
    bg = dev(W.example1_rhs())
    its = {}
    for key, opts, oracle in (
            ("add", dict(method=amg.ADDITIVE_PCG, nu=6), lambda: C.additive_pcg(h, b, 1e-8, 3000, nu=6, omega=0.5)),
            ("v", dict(method=amg.VCYCLE_PCG, nu_pre=3, nu_post=3),
             lambda: C.vcycle_pcg(h, b, 1e-8, 3000, nu_pre=3, nu_post=3, omega=0.5))):
        s = amg.Solver(2, N1, W.EXAMPLE1_LEVELS, stencil=st, omega=0.5, maxit=3000, **opts)
        _, info = s.solve(bg, tol=1e-8)
        _, k_o, _ = oracle()
        assert info["status"] == amg.OK and abs(info["iterations"] - k_o) <= 1, (key, info, k_o)
        its[key] = info["iterations"]
        s.close()
    s = amg.Solver(2, N1, W.EXAMPLE1_LEVELS, stencil=st, **OPTS)
    _, info = s.solve(bg, tol=1e-8)
    its["mpcg"] = info["iterations"]
    s.close()
    assert its["v"] < its["mpcg"] < its["add"], its


def test_example1_mixed_precision():
    s = amg.Solver(2, N1, W.EXAMPLE1_LEVELS, stencil=W.example1_stencil(1e-1), precision=1, **OPTS)
    bg = dev(W.example1_rhs())
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK
    rt = s.residual(bg, x)
    assert float(torch.linalg.norm(rt) / torch.linalg.norm(bg)) <= 1e-8
    s.close()


def test_stencil_setup_validation():
    st = W.example1_stencil(1e-1)
    bad = st.copy()
    bad[0, 0] += 1.0                      # not symmetric
    for kw in (dict(stencil=bad), dict(stencil=-st)):
        with pytest.raises(amg.AmgMpcgError):
            amg.Solver(2, N1, 4, **kw)
    with pytest.raises(amg.AmgMpcgError):
        amg.Solver(3, 15, 2, stencil=st)
