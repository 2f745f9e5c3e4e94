"""Element-wise GPU parity at the benchmarked workload itself: 3D Poisson,
127^3 interior nodes (2,048,383 DoF), 6 levels (b = 6 directions), FP64, in
the launch configuration the benchmark times (default options), against the
FP64 oracle run in the test on the same seeded inputs.

Every node is compared (no sampling), with two bars for a vector v against
the oracle's v_o: normwise ||v - v_o|| <= t ||v_o|| and element-wise
max |v - v_o| <= t max |v_o|.  The element-wise bar catches an error confined
to one grid line or tile edge, which the normwise one dilutes by sqrt(N).

FP64: the level-correction block Z = MG(r) (Algorithm 1, "corrections from
all levels") to 1e-13 per column, iterates x_k at equal k (tol = 0) to
1e-10, the converged iteration count equal or within one.

FP32 bulk (operators, transfers, smoothers and direction blocks in FP32;
x, r, the Gram matrix and its pseudo-inverse in FP64): Z per column against
the FP64 oracle to a bar derived from FP32 rounding (below), and the
converged solution's error against the oracle's FP64 solution, reported and
bounded by the conditioning of A times the tolerance.

The general (CSR) entry point at the same size: Z per column 1e-13 and
x_1 1e-10 against the oracle built from the same matrices, and its
converged iterate equal to the structured path's to 1e-10.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy, mpcg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2402_12833_amd as amg  # noqa: E402

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    amg.load()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def errs(v, vo):
    """(normwise relative, element-wise max relative to max |v_o|)."""
    nv = np.linalg.norm(vo)
    mv = np.abs(vo).max()
    return (np.linalg.norm(v - vo) / (nv if nv > 0 else 1.0),
            np.abs(v - vo).max() / (mv if mv > 0 else 1.0))


def assert_close(v, vo, tol, what):
    e2, einf = errs(v, vo)
    print(f"{what}: normwise {e2:.3e}, element-wise {einf:.3e} (bar {tol:.1e})", flush=True)
    assert e2 <= tol and einf <= tol, (what, e2, einf)


@pytest.fixture(scope="module")
def bench():
    """The 127^3 Poisson workload, its oracle hierarchy and the oracle's
    converged solve with the iterates at k = 1, 2, 5 kept."""
    prob = W.POISSON3D_127
    print(f"oracle: {prob.name}, n={prob.n}, levels={prob.nlevels}", flush=True)
    h = hierarchy.build(prob.dim, prob.n, prob.nlevels)
    b = W.problem_rhs(prob)
    ref = mpcg.mpcg(h, b, tol=1e-8, snapshots=(1, 2, 5))
    print(f"oracle: {ref.iterations} iterations", flush=True)
    return prob, h, b, ref


def test_bench_fp64_mg_block(bench):
    prob, h, b, _ = bench
    s = amg.Solver(prob.dim, prob.n, prob.nlevels)
    Zg = host(s.mg_block(dev(b)))
    Zo = mpcg.mg_block(h, b)
    assert Zg.shape == (prob.nlevels, prob.ndof)
    for l in range(prob.nlevels):
        assert_close(Zg[l], Zo[:, l], 1e-13, f"Z column {l}")
    s.close()


def test_bench_fp64_iterates_full_vector(bench):
    prob, h, b, ref = bench
    s = amg.Solver(prob.dim, prob.n, prob.nlevels)
    bg = dev(b)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and info["nb"] == 6
    assert abs(info["iterations"] - ref.iterations) <= 1, (info["iterations"], ref.iterations)
    if info["iterations"] == ref.iterations:
        assert_close(host(x), ref.x, 1e-10, f"converged x (k = {ref.iterations})")
    for k in (1, 2, 5):
        xg, inf = s.solve(bg, tol=0.0, maxit=k)
        assert inf["iterations"] == k
        assert_close(host(xg), ref.snapshots[k], 1e-10, f"x_{k}")
    xg, _ = s.solve(bg, tol=0.0, maxit=ref.iterations)
    assert_close(host(xg), ref.x, 1e-10, f"x_{ref.iterations} (tol = 0)")
    # residual history of the converged run
    s.solve(bg, tol=1e-8)
    _, res = s.history()
    np.testing.assert_allclose(res[: ref.iterations + 1], ref.resnorms, rtol=1e-8)
    s.close()


def fp32_block_bar(L, l, nu):
    """FP32 rounding bar for column l of Z (relative, normwise and
    element-wise).  The column passes through L - l restrictions, nu
    damped-Jacobi sweeps and L - l prolongations, s = 2(L - l) + nu + 1
    steps counting the rounding of r to FP32.  Each step's output is a sum
    of at most 27 terms rounded to FP32 (unit roundoff u = 2^-24), with
    rounding errors that add like a random walk: about sqrt(27) u ~ 5 u per
    sum.  The terms of restriction and prolongation have positive weights;
    the Jacobi residual g - A c has cancelling ones, but |D^-1||A| has row
    sum 2 on these M-matrices, and the FP32 coefficients of A perturb each
    sweep by about u more.  The bar allows 8 u per step: s * 8 u (5.0e-7 per
    step; a wrong index or a dropped term gives errors of order 1e-3 or
    more)."""
    steps = 2 * (L - l) + nu + 1
    return steps * 8.0 * U32


@pytest.mark.parametrize("case", [(3, 31, 4, None, 17), (3, 31, 4, 3, 18), "bench"],
                         ids=["d3n31L4", "d3n31L4k3", "poisson3d_127"])
def test_fp32_mg_block(case, bench):
    if case == "bench":
        prob, h, b, _ = bench
        dim, n, nl = prob.dim, prob.n, prob.nlevels
        kap = None
    else:
        dim, n, nl, ks, seed = case
        prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
        kap = W.kappa_field(prob)
        h = hierarchy.build(dim, n, nl, kappa=kap)
        b = W.rhs(n ** dim, seed)
    s = amg.Solver(dim, n, nl, kappa=kap, precision=1)
    Zg = host(s.mg_block(dev(b)))
    Zo = mpcg.mg_block(h, b)
    L = nl - 1
    for l in range(nl):
        assert_close(Zg[l], Zo[:, l], fp32_block_bar(L, l, 2), f"FP32 Z column {l}")
    s.close()


def test_bench_fp32_solution_error(bench):
    """X1: the FP32-bulk solve reaches a true FP64 relative residual <= 1e-8
    with at most a few more iterations than the FP64 oracle, and its error
    against the oracle's FP64 solution (reported) is within what the
    tolerance allows: both solutions have relative residual <= 1e-8, so
    their difference is at most 2 * cond(A) * 1e-8 relative, cond(A) of the
    127^3 Laplacian = cot^2(pi h / 2) ~ 6.6e3."""
    prob, h, b, ref = bench
    s = amg.Solver(prob.dim, prob.n, prob.nlevels, precision=1)
    bg = dev(b)
    x, info = s.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK
    xh = host(x)
    true_rel = np.linalg.norm(b - h.fine.A @ xh) / np.linalg.norm(b)
    e2, einf = errs(xh, ref.x)
    hh = 1.0 / (prob.n + 1)
    cond = 1.0 / np.tan(np.pi * hh / 2) ** 2
    print(f"FP32 bulk {prob.name}: {info['iterations']} iterations (FP64 oracle {ref.iterations}), "
          f"{info['refreshes']} refreshes, true relres {true_rel:.3e}, "
          f"error vs FP64 oracle normwise {e2:.3e}, element-wise {einf:.3e}", flush=True)
    assert true_rel <= 1e-8
    assert info["iterations"] <= ref.iterations + 2
    assert e2 <= 2.0 * cond * 1e-8
    s.close()


def test_bench_csr_entry_point(bench):
    """The same workload through the general entry point (the fine 7-point
    operator as a 14,241,907-entry CSR matrix, the trilinear prolongations
    as CSR, R = 2^-3 P^T)."""
    prob, h, b, ref = bench
    Ps = [h.levels[l].P for l in range(prob.nlevels - 1)]
    A = h.fine.A.tocsr()
    ho = hierarchy.from_operators(A, Ps, 0.125)
    c = amg.Solver.from_csr(A, Ps, 0.125)
    bg = dev(b)
    Zg = host(c.mg_block(bg))
    Zo = mpcg.mg_block(ho, b)
    for l in range(prob.nlevels):
        assert_close(Zg[l], Zo[:, l], 1e-13, f"CSR Z column {l}")
    x1, _ = c.solve(bg, tol=0.0, maxit=1)
    assert_close(host(x1), mpcg.mpcg(ho, b, tol=0.0, maxit=1).x, 1e-10, "CSR x_1")
    x, info = c.solve(bg, tol=1e-8)
    assert info["status"] == amg.OK and abs(info["iterations"] - ref.iterations) <= 1
    g = amg.Solver(prob.dim, prob.n, prob.nlevels)
    xs, infos = g.solve(bg, tol=1e-8)
    assert info["iterations"] == infos["iterations"]
    assert_close(host(x), host(xs), 1e-10, "CSR vs structured converged x")
    g.close()
    c.close()
