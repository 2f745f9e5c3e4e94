"""C-ABI library: loads, exports every declared symbol, validates arguments
on the host before any device work (no GPU needed for these checks)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import paper_2402_12833_amd as amg
from paper_2402_12833_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2402_12833_amd import build
        build.build()
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = B.header_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_default_options(lib):
    o = amg.default_options()
    assert (o.m, o.nu, o.maxit, o.precision, o.k_poll) == (1, 2, 1000, 0, 8)
    assert o.true_residual == 1
    assert o.omega == pytest.approx(2.0 / 3.0)
    assert o.refresh_drop == pytest.approx(1e-2)


def _setup(lib, grid, opts):
    h = ctypes.c_void_p()
    code = lib.amgmpcg_setup_grid(ctypes.byref(grid) if grid is not None else None,
                                  ctypes.byref(opts) if opts is not None else None, None, ctypes.byref(h))
    return code, h


@pytest.mark.parametrize("grid,expect", [
    (B.Grid(4, 31, 3, None), B.INVALID_ARG),     # dim
    (B.Grid(2, 0, 1, None), B.INVALID_ARG),      # n
    (B.Grid(2, 31, 0, None), B.INVALID_ARG),     # levels
    (B.Grid(2, 31, 9, None), B.INVALID_ARG),     # too many directions
    (B.Grid(2, 7, 4, None), B.DIM_MISMATCH),     # 7 -> 3 -> 1 -> 0
])
def test_grid_validation(lib, grid, expect):
    code, h = _setup(lib, grid, amg.default_options())
    assert code == expect
    assert not h.value
    assert B.last_error()


@pytest.mark.parametrize("kw", [dict(m=0), dict(m=9), dict(nu=0), dict(omega=1.5), dict(maxit=0), dict(precision=3),
                                dict(k_poll=0), dict(refresh_drop=2.0), dict(method=3), dict(method=-1),
                                dict(method=1, m=2), dict(method=2, nu_pre=1, nu_post=2), dict(nu_pre=9, nu_post=9),
                                dict(true_residual=2), dict(true_residual=-1)])
def test_option_validation(lib, kw):
    code, _ = _setup(lib, B.Grid(2, 31, 3, None), amg.default_options(**kw))
    assert code == B.INVALID_ARG


def test_kappa_validation(lib):
    n = 7
    kap = np.ones((n + 2) ** 2)
    kap[10] = np.nan
    g = B.Grid(2, n, 2, kap.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert _setup(lib, g, amg.default_options())[0] == B.NONFINITE
    kap[10] = -1.0
    assert _setup(lib, g, amg.default_options())[0] == B.NOT_SPD


def test_null_arguments(lib):
    assert _setup(lib, None, amg.default_options())[0] == B.INVALID_ARG
    assert _setup(lib, B.Grid(2, 31, 3, None), None)[0] == B.INVALID_ARG
    info = B.Info()
    assert lib.amgmpcg_solve(None, None, None, 1e-8, 0, ctypes.byref(info)) == B.INVALID_ARG
    assert lib.amgmpcg_mg_block(None, None, None) == B.INVALID_ARG
    v = ctypes.c_int64(-1)
    assert lib.amgmpcg_workspace_bytes(None, ctypes.byref(v)) == B.INVALID_ARG and v.value == -1
    lib.amgmpcg_destroy(None)


def test_status_strings(lib):
    for c in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert B.status_string(c) and B.status_string(c) != "unknown status"
    assert B.status_string(99) == "unknown status"


def test_stencil_setup_validation(lib):
    """Argument checks of the 9-point-stencil setup (before any device call)."""
    h = ctypes.c_void_p()
    st = np.array([-1.0, -4.0, -1.0, 2.0, 8.0, 2.0, -1.0, -4.0, -1.0]) / 6.0
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    asym = st.copy()
    asym[0] += 1.0
    nan = st.copy()
    nan[2] = nan[6] = np.nan
    kap = np.ones(33 * 33)
    cases = [
        (B.Grid(3, 15, 2, None), st, B.INVALID_ARG),
        (B.Grid(2, 31, 3, dp(kap)), st, B.INVALID_ARG),
        (B.Grid(2, 31, 3, None), asym, B.INVALID_ARG),
        (B.Grid(2, 31, 3, None), -st, B.NOT_SPD),
        (B.Grid(2, 31, 3, None), nan, B.NONFINITE),
    ]
    for g, w, want in cases:
        code = lib.amgmpcg_setup_stencil(ctypes.byref(g), dp(np.ascontiguousarray(w)),
                                         ctypes.byref(amg.default_options()), None, ctypes.byref(h))
        assert code == want and not h.value, (want, code)
    assert lib.amgmpcg_setup_stencil(ctypes.byref(B.Grid(2, 31, 3, None)), None,
                                     ctypes.byref(amg.default_options()), None, ctypes.byref(h)) == B.INVALID_ARG


def test_csr_setup_validation(lib):
    """Argument checks of the CSR setup (before any device call)."""
    import scipy.sparse as sp
    h = ctypes.c_void_p()
    A = sp.diags([np.full(8, -1.0), np.full(9, 2.0), np.full(8, -1.0)], [-1, 0, 1]).tocsr()
    P = sp.csr_matrix((np.ones(9), (np.arange(9), np.arange(9) // 3)), shape=(9, 3))

    def setup(Am, Pm=None, nl=2, scale=1.0, **kw):
        keep = []
        a = B._csr_struct(Am, keep)
        arr = (B.CsrMatrix * 1)()
        if Pm is not None:
            arr[0] = B._csr_struct(Pm, keep)
        H = B.Hierarchy(nl, arr if Pm is not None else None, scale)
        return lib.amgmpcg_setup_csr(ctypes.byref(a), ctypes.byref(H), ctypes.byref(amg.default_options(**kw)),
                                     None, ctypes.byref(h))

    nonsym = A.tolil()
    nonsym[0, 1] = -2.0
    nan = A.copy()
    nan.data[3] = np.nan
    badP = sp.csr_matrix((np.ones(8), (np.arange(8), np.arange(8) // 3)), shape=(8, 3))
    assert setup(A[:, :8], P) == B.INVALID_ARG                      # not square
    assert setup(nonsym.tocsr(), P) == B.NOT_SPD                     # not symmetric
    assert setup(nan, P) == B.NONFINITE
    assert setup(A, badP) == B.INVALID_ARG                           # P rows != unknowns
    assert setup(A, P, scale=0.0) == B.INVALID_ARG
    assert setup(A, None, nl=2) == B.INVALID_ARG                     # prolongations missing
    assert setup(A, P, method=1) == B.INVALID_ARG
    keep = []
    a = B._csr_struct(A, keep)
    keep[0][3] = 99                                                  # corrupt row pointers
    H = B.Hierarchy(1, None, 1.0)
    assert lib.amgmpcg_setup_csr(ctypes.byref(a), ctypes.byref(H), ctypes.byref(amg.default_options()), None,
                                 ctypes.byref(h)) == B.INVALID_ARG
    keep = []
    a = B._csr_struct(A, keep)
    keep[1][0] = 40                                                  # column out of range
    assert lib.amgmpcg_setup_csr(ctypes.byref(a), ctypes.byref(H), ctypes.byref(amg.default_options()), None,
                                 ctypes.byref(h)) == B.INVALID_ARG
    assert not h.value


def test_batched_validation(lib):
    """Argument checks of the batched entry point (before any device call)."""
    h = ctypes.c_void_p()
    ok = (B.Grid * 2)(B.Grid(2, 31, 3, None), B.Grid(2, 15, 2, None))
    kap = np.ones(33 * 33)
    cases = [
        (1, (B.Grid * 1)(B.Grid(2, 31, 3, kap.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))), {}),
        (2, (B.Grid * 2)(B.Grid(2, 31, 3, None), B.Grid(3, 15, 2, None)), {}),
        (1, (B.Grid * 1)(B.Grid(2, 255, 7, None)), {}),
        (2, ok, dict(nu=3)),
        (2, ok, dict(m=2)),
        (2, ok, dict(method=1)),
        (0, ok, {}),
    ]
    for count, grids, kw in cases:
        code = lib.amgmpcg_setup_batched(count, grids, ctypes.byref(amg.default_options(**kw)), None, ctypes.byref(h))
        assert code == B.INVALID_ARG and not h.value, (count, kw)


def test_cnn_weight_count_matches_the_oracle_layers(lib):
    from oracle import cnn
    total = sum((27 if k == 3 else 1) * cin * cout for _, k, cin, cout in cnn.LAYERS)
    assert amg.cnn_weight_count() == total
    assert [(n, cin, cout) for n, _, cin, cout in B.CNN_LAYERS] == [(n, cin, cout) for n, _, cin, cout in cnn.LAYERS]


def test_cnn_argument_validation(lib):
    h = ctypes.c_void_p()
    assert lib.amgmpcg_cnn_create(0, 0, None, ctypes.byref(h)) == B.INVALID_ARG and not h.value
    assert lib.amgmpcg_cnn_create(1001, 0, None, ctypes.byref(h)) == B.INVALID_ARG and not h.value
    assert lib.amgmpcg_cnn_create(15, 0, None, None) == B.INVALID_ARG
    w = np.zeros(amg.cnn_weight_count(), dtype=np.float32)
    fp = w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    assert lib.amgmpcg_cnn_set_weights(None, fp, w.size) == B.INVALID_ARG
    assert lib.amgmpcg_cnn_get_weights(None, fp, w.size) == B.INVALID_ARG
    assert lib.amgmpcg_cnn_forward(None, None, None, None) == B.INVALID_ARG
    loss = ctypes.c_double()
    assert lib.amgmpcg_cnn_train_step(None, None, None, None, 1e-3, ctypes.byref(loss)) == B.INVALID_ARG
    assert lib.amgmpcg_attach_cnn(None, None) == B.INVALID_ARG
    assert lib.amgmpcg_log_kappa(None, None) == B.INVALID_ARG
    assert lib.amgmpcg_residual(None, None, None, None) == B.INVALID_ARG
    ks = (ctypes.c_int32 * 1)(0)
    assert lib.amgmpcg_make_pairs(None, None, None, ks, 1, None, None) == B.INVALID_ARG
    lib.amgmpcg_cnn_destroy(None)


def test_bind_workspace_null_handle(lib):
    """The workspace entry points reject a missing handle on the host."""
    buf = ctypes.create_string_buffer(1024)
    assert lib.amgmpcg_bind_workspace(None, ctypes.cast(buf, ctypes.c_void_p), 1024) == B.INVALID_ARG
    v = ctypes.c_int64()
    assert lib.amgmpcg_workspace_bytes(None, ctypes.byref(v)) == B.INVALID_ARG


def test_info_layout(lib):
    """The info struct carries the true residual and the setup time after the
    fields of the first layout (offsets of a plain C struct)."""
    names = [f for f, _ in B.Info._fields_]
    assert names[-2:] == ["relres_true", "setup_ms"]
    assert B.Info.relres_true.offset == B.Info.solve_ms.offset + 8
    assert ctypes.sizeof(B.Info) == B.Info.setup_ms.offset + 8
