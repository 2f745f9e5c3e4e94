"""GPU parity of the general (CSR) entry point against the FP64 oracle on
the same matrices: the oracle builds its own Galerkin hierarchy from the
given A and prolongations (``hierarchy.from_operators``), the library its
own on the host.

Bars as for the structured path: the level-correction block Z to 1e-13
per column, iterates at equal k to 1e-10 relative, converged counts within
one, FP32 bulk true residual <= 1e-8.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy, mpcg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_12833_amd as amg  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    amg.load()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def rel(a, b):
    """max(normwise, element-wise max |a - b| / max |b|) relative error."""
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


def structured_case(dim, n, nl, ks, seed):
    prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
    h = hierarchy.build(dim, n, nl, kappa=W.kappa_field(prob))
    Ps = [h.levels[l].P for l in range(nl - 1)]
    return h.fine.A, Ps, 0.5 ** dim, W.rhs(n ** dim, seed)


def graph_case(npts, seed, nl):
    A, Ps, b = W.graph_problem(npts=npts, seed=seed, nlevels=nl)
    return A, Ps, 1.0, b


CASES = {
    "fd2d_31": lambda: structured_case(2, 31, 4, None, 1),
    "fd3d_17_kappa": lambda: structured_case(3, 17, 3, 3, 15),
    "graph_4000": lambda: graph_case(4000, 11, 4),
    "graph_1500_2lev": lambda: graph_case(1500, 12, 2),
    "graph_500_1lev": lambda: graph_case(500, 13, 1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_csr_iterates_match_oracle(name):
    A, Ps, scale, b = CASES[name]()
    h = hierarchy.from_operators(A, Ps, scale)
    s = amg.Solver.from_csr(A, Ps, scale, maxit=3000)
    bg = dev(b)
    Z = s.mg_block(bg).cpu().numpy()
    Zo = mpcg.mg_block(h, b)
    for l in range(len(Ps) + 1):
        assert rel(Z[l], Zo[:, l]) <= 1e-13, l
    ref = mpcg.mpcg(h, b, tol=1e-8, maxit=3000)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and abs(info["iterations"] - ref.iterations) <= 1, (info, ref.iterations)
    for k in sorted({1, 5, min(30, ref.iterations)}):
        o = mpcg.mpcg(h, b, tol=0.0, maxit=k)
        xg, inf = s.solve(bg, tol=0.0, maxit=k)
        assert rel(xg.cpu().numpy(), o.x) <= 1e-10, (k, rel(xg.cpu().numpy(), o.x))
    rt = s.residual(bg, x)
    assert float(torch.linalg.norm(rt) / torch.linalg.norm(bg)) <= 1.01e-8
    s.close()


@pytest.mark.parametrize("opts", [dict(m=5), dict(nu=3), dict(nu=4, omega=0.5)], ids=["m5", "nu3", "nu4"])
def test_csr_options_match_oracle(opts):
    A, Ps, scale, b = graph_case(3000, 21, 3)
    h = hierarchy.from_operators(A, Ps, scale)
    s = amg.Solver.from_csr(A, Ps, scale, maxit=3000, **opts)
    bg = dev(b)
    oo = {k: v for k, v in opts.items()}
    for k in (1, 7, 25):
        o = mpcg.mpcg(h, b, tol=0.0, maxit=k, **oo)
        xg, _ = s.solve(bg, tol=0.0, maxit=k)
        assert rel(xg.cpu().numpy(), o.x) <= 1e-10, (opts, k)
    ref = mpcg.mpcg(h, b, tol=1e-8, maxit=3000, **oo)
    _, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and abs(info["iterations"] - ref.iterations) <= 1
    s.close()


@pytest.mark.parametrize("nu", [4, 6])
def test_csr_even_sweep_counts_repeatable(nu):
    """With an even number of sweeps the smoother's last pass reads the
    second scratch vector; it must never be the output itself (an in-place
    Jacobi pass races between rows).  Repeated solves agree bit for bit."""
    for nl in (1, 3):
        A, Ps, scale, b = graph_case(3000, 21, nl)
        s = amg.Solver.from_csr(A, Ps, scale, maxit=3000, nu=nu)
        rhs = dev(b)
        ref = s.solve(rhs, tol=0.0, maxit=12)[0].cpu().numpy()
        for _ in range(4):
            assert np.array_equal(s.solve(rhs, tol=0.0, maxit=12)[0].cpu().numpy(), ref), (nu, nl)
        Z0 = s.mg_block(rhs).cpu().numpy()
        for _ in range(8):
            assert np.array_equal(s.mg_block(rhs).cpu().numpy(), Z0), (nu, nl)
        s.close()


def test_csr_mixed_precision():
    A, Ps, scale, b = graph_case(4000, 11, 4)
    s = amg.Solver.from_csr(A, Ps, scale, precision=1, maxit=3000)
    bg = dev(b)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK
    rt = s.residual(bg, x)
    assert float(torch.linalg.norm(rt) / torch.linalg.norm(bg)) <= 1e-8
    s.close()


def test_csr_matches_structured_path():
    """The same 3D problem through both entry points: equal iterates to 1e-10."""
    A, Ps, scale, b = structured_case(3, 31, 4, None, 17)
    c = amg.Solver.from_csr(A, Ps, scale)
    g = amg.Solver(3, 31, 4)
    bg = dev(b)
    for k in (3, 10):
        xc, _ = c.solve(bg, tol=0.0, maxit=k)
        xs, _ = g.solve(bg, tol=0.0, maxit=k)
        assert rel(xc.cpu().numpy(), xs.cpu().numpy()) <= 1e-10
    c.close()
    g.close()


def test_csr_handle_restrictions():
    A, Ps, scale, b = graph_case(500, 13, 2)
    s = amg.Solver.from_csr(A, Ps, scale)
    assert s.workspace_bytes() > A.nnz * 12
    with pytest.raises(amg.AmgMpcgError):
        s.level_stencil(0)
    s.close()
