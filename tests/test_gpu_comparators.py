"""GPU parity of the comparison methods of Sec. 3 (additive MG-PCG and
MG(V)-PCG, through the C ABI) against the oracle's textbook PCG with the
same preconditioners.

The GPU runs CG in the A-orthogonalisation form of the MPCG machinery with
one direction, the oracle in the Hestenes-Stiefel form; the two agree in
exact arithmetic.  Bars: iterates x_k at equal k to 1e-10 relative for
k <= 5 and 1e-8 at the converged count (the two recurrences round
differently), converged iteration counts within one, residual norms to
1e-6 relative; FP32 bulk: true FP64 relative residual <= 1e-8.
"""
import numpy as np
import pytest

import workloads as W
from oracle import comparators as C
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


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """max(normwise, element-wise max |a - b| / max |b|) relative error."""
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    return max(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0),
               (np.abs(a - b).max() / mb) if mb > 0 else 0.0)


CASES = [
    (2, 31, 4, None, 1),
    (2, 45, 4, 5, 12),
    (2, 20, 2, None, 14),
    (3, 17, 3, None, 15),
    (3, 15, 3, 3, 16),
    (3, 31, 4, None, 17),
    (3, 13, 1, None, 18),
]
METHODS = {amg.ADDITIVE_PCG: "additive", amg.VCYCLE_PCG: "vcycle"}


def case_id(c):
    return f"d{c[0]}n{c[1]}L{c[2]}k{c[3]}"


def oracle_pcg(method, h, b, **kw):
    if method == amg.ADDITIVE_PCG:
        return C.additive_pcg(h, b, **kw)
    return C.vcycle_pcg(h, b, **kw)


def build(dim, n, nl, ks, seed, method, **opts):
    prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
    kap = W.kappa_field(prob)
    h = hierarchy.build(dim, n, nl, kappa=kap)
    s = amg.Solver(dim, n, nl, kappa=kap, method=method, **opts)
    return h, s, W.rhs(n ** dim, seed)


@pytest.mark.parametrize("case", CASES, ids=case_id)
@pytest.mark.parametrize("method", list(METHODS), ids=list(METHODS.values()))
def test_iterates_match_oracle_pcg(case, method):
    h, s, b = build(*case, method)
    x_o, k_o, hist = oracle_pcg(method, h, b, tol=1e-8)
    bg = dev(b)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and info["nb"] == 1
    assert abs(info["iterations"] - k_o) <= 1, (info["iterations"], k_o)
    for kk in sorted({1, 2, min(5, k_o), k_o}):
        xo, _, _ = oracle_pcg(method, h, b, tol=0.0, maxit=kk)
        xg, inf = s.solve(bg, tol=0.0, maxit=kk)
        assert inf["iterations"] == kk
        bar = 1e-10 if kk <= 5 else 1e-8
        assert rel(host(xg), xo) <= bar, (kk, rel(host(xg), xo))
    s.solve(bg, tol=1e-8)
    alph, res = s.history()
    m = min(len(res), len(hist))
    np.testing.assert_allclose(res[:m], hist[:m], rtol=1e-6)
    s.close()


@pytest.mark.parametrize("case", [CASES[0], CASES[4], CASES[5]], ids=case_id)
@pytest.mark.parametrize("method", list(METHODS), ids=list(METHODS.values()))
def test_mixed_precision_reaches_tolerance(case, method):
    h, s, b = build(*case, method, precision=1)
    _, k_o, _ = oracle_pcg(method, h, b, tol=1e-8)
    bg = dev(b)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK
    rt = s.residual(bg, x)
    assert float(torch.linalg.norm(rt) / torch.linalg.norm(bg)) <= 1e-8
    assert info["iterations"] <= k_o + 2
    s.close()


@pytest.mark.parametrize("method", list(METHODS), ids=list(METHODS.values()))
def test_full_size_poisson(method):
    prob = W.POISSON3D_127
    h = hierarchy.build(prob.dim, prob.n, prob.nlevels)
    b = W.problem_rhs(prob)
    s = amg.Solver(prob.dim, prob.n, prob.nlevels, method=method)
    bg = dev(b)
    xo, _, _ = oracle_pcg(method, h, b, tol=0.0, maxit=3)
    xg, inf = s.solve(bg, tol=0.0, maxit=3)
    assert rel(host(xg), xo) <= 1e-10
    _, k_o, _ = oracle_pcg(method, h, b, tol=1e-8)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and abs(info["iterations"] - k_o) <= 1
    s.close()


def test_paper_ordering_on_the_gpu():
    """Sec. 3 on a heterogeneous 3D case: V-cycle PCG < MPCG (m = 5) <
    additive MG-PCG in iterations, as the oracle has it."""
    dim, n, nl, ks, seed = 3, 31, 4, 3, 4
    its = {}
    for key, opts in (("v", dict(method=amg.VCYCLE_PCG)), ("mp", dict(m=5)), ("add", dict(method=amg.ADDITIVE_PCG))):
        prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
        s = amg.Solver(dim, n, nl, kappa=W.kappa_field(prob), **opts)
        _, info = s.solve(dev(W.rhs(n ** dim, seed)), tol=1e-8)
        assert info["status"] == amg.OK
        its[key] = info["iterations"]
        s.close()
    assert its["v"] < its["mp"] < its["add"], its


def test_comparison_method_restrictions():
    s = amg.Solver(2, 31, 4, method=amg.ADDITIVE_PCG)
    with pytest.raises(amg.AmgMpcgError):
        s.mg_block(dev(np.ones(31 * 31)))
    s.close()
    for bad in (dict(method=3), dict(method=amg.VCYCLE_PCG, m=2), dict(method=amg.VCYCLE_PCG, nu_pre=1, nu_post=2)):
        with pytest.raises(amg.AmgMpcgError):
            amg.Solver(2, 31, 4, **bad)
