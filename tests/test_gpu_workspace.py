"""The boundary's workspace and reporting entry points on the GPU: a handle
whose buffers are routed through a torch-owned workspace
(amgmpcg_bind_workspace) computes bit for bit what a self-allocated handle
computes, can be bound again, and rejects unusable memory on the host; the
true residual and the setup time reported in amgmpcg_info."""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy

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


def grid_pair(dim, n, nl, ks, seed, **opts):
    prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
    kap = W.kappa_field(prob)
    mk = lambda: amg.Solver(dim, n, nl, kappa=kap, **opts)  # noqa: E731
    return mk(), mk(), W.rhs(n ** dim, seed)


def csr_pair(**opts):
    A, Ps, b = W.graph_problem(npts=3000, seed=21, nlevels=3)
    mk = lambda: amg.Solver.from_csr(A, Ps, 1.0, **opts)  # noqa: E731
    return mk(), mk(), b


CASES = {
    "d3n31L4": lambda: grid_pair(3, 31, 4, None, 17),
    "d3n31L4k3_fp32": lambda: grid_pair(3, 31, 4, 3, 18, precision=1),
    "d3n31L4k3_m5": lambda: grid_pair(3, 31, 4, 3, 18, m=5),
    "d2n45L4k5": lambda: grid_pair(2, 45, 4, 5, 12),
    "d2n31L4_vcycle": lambda: grid_pair(2, 31, 4, None, 1, method=amg.VCYCLE_PCG),
    "csr_graph": lambda: csr_pair(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_bound_workspace_is_bit_identical(name):
    own, bound, b = CASES[name]()
    bg = dev(b)
    need = bound.workspace_bytes()
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    bound.bind_workspace(ws)
    assert bound.workspace_bytes() == need
    x1, i1 = own.solve(bg, tol=1e-8)
    x2, i2 = bound.solve(bg, tol=1e-8)
    assert i1["status"] == i2["status"] == amg.OK
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x2)
    a1, r1 = own.history()
    a2, r2 = bound.history()
    assert np.array_equal(a1, a2) and np.array_equal(r1, r2)
    if name != "d2n31L4_vcycle":
        assert torch.equal(own.mg_block(bg), bound.mg_block(bg))
    # bound again into a second region; the first can then be released
    ws2 = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    bound.bind_workspace(ws2)
    del ws
    torch.cuda.synchronize()
    x3, i3 = bound.solve(bg, tol=0.0, maxit=3)
    x4, _ = own.solve(bg, tol=0.0, maxit=3)
    assert torch.equal(x3, x4)
    own.close()
    bound.close()


def test_bind_workspace_rejects_unusable_memory():
    s, _, b = grid_pair(3, 15, 3, None, 16)
    need = s.workspace_bytes()
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(amg.AmgMpcgError) as e:
        s.bind_workspace(small)
    assert e.value.code == amg.INVALID_ARG
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(amg.AmgMpcgError) as e:
        s.bind_workspace(big[1:])        # not 256-byte aligned
    assert e.value.code == amg.INVALID_ARG
    host = np.zeros(need + 512, dtype=np.uint8)
    addr = (host.ctypes.data + 255) // 256 * 256
    code = s._lib.amgmpcg_bind_workspace(s._h, amg.binding.c_void_p(addr), need)
    assert code == amg.INVALID_ARG
    # the handle is unchanged by the refusals and still solves
    x, info = s.solve(dev(b), tol=1e-8)
    assert info["status"] == amg.OK
    # bound: attaching a network is refused (it would grow the blocks)
    s.bind_workspace()
    net = amg.Network(15)
    with pytest.raises(amg.AmgMpcgError) as e:
        s.attach(net)
    assert e.value.code == amg.INVALID_ARG
    net.close()
    bs = amg.BatchedSolver([(2, 31, 3), (2, 15, 2)])
    code = bs._lib.amgmpcg_bind_workspace(bs._h, amg.binding.c_void_p(big.data_ptr()), need)
    assert code == amg.INVALID_ARG
    bs.close()
    s.close()


@pytest.mark.parametrize("case,precision", [((3, 31, 4, None, 17), 0), ((3, 31, 4, 3, 18), 0),
                                            ((3, 31, 4, 3, 18), 1), ((2, 31, 4, None, 1), 0)])
def test_info_true_residual_and_setup_time(case, precision):
    dim, n, nl, ks, seed = case
    prob = W.GridProblem("t", dim, n, nl, seed, kappa_seed=ks)
    kap = W.kappa_field(prob)
    h = hierarchy.build(dim, n, nl, kappa=kap)
    b = W.rhs(n ** dim, seed)
    s = amg.Solver(dim, n, nl, kappa=kap, precision=precision)
    x, info = s.solve(dev(b), tol=1e-8)
    xh = x.cpu().numpy()
    true_rel = np.linalg.norm(b - h.fine.A @ xh) / np.linalg.norm(b)
    assert abs(info["relres_true"] - true_rel) <= 1e-4 * true_rel
    assert info["relres_true"] <= 1.01e-8
    assert info["setup_ms"] > 0.0
    off = amg.Solver(dim, n, nl, kappa=kap, precision=precision, true_residual=0)
    x2, info2 = off.solve(dev(b), tol=1e-8)
    assert info2["relres_true"] == -1.0
    assert torch.equal(x, x2)
    s.close()
    off.close()


def test_info_true_residual_csr():
    A, Ps, b = W.graph_problem(npts=3000, seed=21, nlevels=3)
    s = amg.Solver.from_csr(A, Ps, 1.0)
    x, info = s.solve(dev(b), tol=1e-8)
    true_rel = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
    assert abs(info["relres_true"] - true_rel) <= 1e-4 * true_rel
    assert info["setup_ms"] > 0.0
    s.close()
