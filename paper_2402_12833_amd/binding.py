"""ctypes binding of libamgmpcg.so (argument marshalling only).

Every step of the solver runs in the library's HIP kernels; PyTorch is used
only to own device memory and to supply the current HIP stream.  If the
shared library is missing the binding raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_double, c_int32, c_void_p
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamgmpcg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "amgmpcg.h")

OK, MAXIT, BREAKDOWN = 0, 1, 2
# solution methods (Solver(..., method=...))
MPCG, ADDITIVE_PCG, VCYCLE_PCG = 0, 1, 2
INVALID_ARG, NOT_SPD, DIM_MISMATCH, NONFINITE, OOM, HIP_ERROR, UNAVAILABLE = -1, -2, -3, -4, -5, -6, -7


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n", c_int32), ("nlevels", c_int32), ("kappa", POINTER(c_double))]


class Options(ctypes.Structure):
    _fields_ = [("m", c_int32), ("nu", c_int32), ("omega", c_double), ("maxit", c_int32),
                ("precision", c_int32), ("pinv_tau", c_double), ("k_poll", c_int32),
                ("record_history", c_int32), ("refresh_drop", c_double), ("method", c_int32),
                ("nu_pre", c_int32), ("nu_post", c_int32), ("true_residual", c_int32),
                ("persistent", c_int32)]


class CsrMatrix(ctypes.Structure):
    _fields_ = [("nrows", c_int32), ("ncols", c_int32), ("nnz", c_int32), ("rowptr", POINTER(c_int32)),
                ("colind", POINTER(c_int32)), ("val", POINTER(c_double))]


class Hierarchy(ctypes.Structure):
    _fields_ = [("nlevels", c_int32), ("P", POINTER(CsrMatrix)), ("restrict_scale", c_double)]


def _csr_struct(M, keep: list) -> CsrMatrix:
    """A scipy.sparse matrix as a CsrMatrix over arrays kept alive in `keep`."""
    import scipy.sparse as sp
    M = sp.csr_matrix(M)
    ptr = np.ascontiguousarray(M.indptr, dtype=np.int32)
    col = np.ascontiguousarray(M.indices, dtype=np.int32)
    val = np.ascontiguousarray(M.data, dtype=np.float64)
    keep.extend([ptr, col, val])
    return CsrMatrix(M.shape[0], M.shape[1], int(val.size), ptr.ctypes.data_as(POINTER(c_int32)),
                     col.ctypes.data_as(POINTER(c_int32)), val.ctypes.data_as(POINTER(c_double)))


class Info(ctypes.Structure):
    _fields_ = [("status", c_int32), ("iterations", c_int32), ("bnorm", c_double), ("relres", c_double),
                ("refreshes", c_int32), ("nb", c_int32), ("solve_ms", c_double), ("relres_true", c_double),
                ("setup_ms", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AmgMpcgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"amgmpcg error {code}: {msg}")
        self.code = code


_lib = None


def header_functions():
    """Names of the functions declared in include/amgmpcg.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amgmpcg_[a-z_0-9]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2402_12833_amd.build.build()")
    try:
        # torch owns the device memory and streams: let it bring up the HIP
        # runtime first, so that the library binds to the same runtime
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    lib.amgmpcg_default_options.argtypes = [POINTER(Options)]
    lib.amgmpcg_default_options.restype = None
    lib.amgmpcg_setup_grid.argtypes = [POINTER(Grid), POINTER(Options), c_void_p, POINTER(c_void_p)]
    lib.amgmpcg_setup_stencil.argtypes = [POINTER(Grid), POINTER(c_double), POINTER(Options), c_void_p,
                                          POINTER(c_void_p)]
    lib.amgmpcg_setup_stencil.restype = c_int32
    lib.amgmpcg_setup_csr.argtypes = [POINTER(CsrMatrix), POINTER(Hierarchy), POINTER(Options), c_void_p,
                                      POINTER(c_void_p)]
    lib.amgmpcg_setup_csr.restype = c_int32
    lib.amgmpcg_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int32, POINTER(Info)]
    lib.amgmpcg_solve_host.argtypes = [c_void_p, POINTER(c_double), POINTER(c_double), c_double, c_int32,
                                       POINTER(Info)]
    lib.amgmpcg_mg_block.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.amgmpcg_level_count.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_int32)]
    lib.amgmpcg_level_size.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    lib.amgmpcg_level_stencil.argtypes = [c_void_p, c_int32, POINTER(c_double)]
    lib.amgmpcg_history.argtypes = [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), POINTER(c_int32)]
    lib.amgmpcg_time_kernels.argtypes = [c_void_p, c_int32, POINTER(c_double), c_int32, POINTER(c_int32)]
    lib.amgmpcg_time_kernels.restype = c_int32
    lib.amgmpcg_profile_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int32, POINTER(Info),
                                          POINTER(c_double), c_int32, POINTER(c_int32), POINTER(c_int32)]
    lib.amgmpcg_profile_solve.restype = c_int32
    lib.amgmpcg_setup_batched.argtypes = [c_int32, POINTER(Grid), POINTER(Options), c_void_p, POINTER(c_void_p)]
    lib.amgmpcg_setup_batched.restype = c_int32
    lib.amgmpcg_solve_batched.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int32, POINTER(Info),
                                          POINTER(c_double)]
    lib.amgmpcg_solve_batched.restype = c_int32
    lib.amgmpcg_batched_size.argtypes = [c_void_p, POINTER(c_int32), POINTER(ctypes.c_int64)]
    lib.amgmpcg_batched_size.restype = c_int32
    lib.amgmpcg_workspace_bytes.argtypes = [c_void_p, POINTER(ctypes.c_int64)]
    lib.amgmpcg_workspace_bytes.restype = c_int32
    lib.amgmpcg_bind_workspace.argtypes = [c_void_p, c_void_p, ctypes.c_int64]
    lib.amgmpcg_bind_workspace.restype = c_int32
    lib.amgmpcg_gram_pinv.argtypes = [POINTER(c_double), c_int32, c_double, POINTER(c_double), POINTER(c_int32)]
    lib.amgmpcg_gram_pinv.restype = c_int32
    lib.amgmpcg_gram_pinv_noalloc.argtypes = [POINTER(c_double), c_int32, c_double, POINTER(c_double),
                                              POINTER(c_int32)]
    lib.amgmpcg_gram_pinv_noalloc.restype = c_int32
    lib.amgmpcg_destroy.argtypes = [c_void_p]
    lib.amgmpcg_destroy.restype = None
    lib.amgmpcg_status_string.argtypes = [c_int32]
    lib.amgmpcg_status_string.restype = ctypes.c_char_p
    lib.amgmpcg_last_error.argtypes = []
    lib.amgmpcg_last_error.restype = ctypes.c_char_p
    lib.amgmpcg_residual.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.amgmpcg_cnn_weight_count.argtypes = []
    lib.amgmpcg_cnn_weight_count.restype = ctypes.c_int64
    lib.amgmpcg_cnn_create.argtypes = [c_int32, ctypes.c_uint64, c_void_p, POINTER(c_void_p)]
    lib.amgmpcg_cnn_set_weights.argtypes = [c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]
    lib.amgmpcg_cnn_get_weights.argtypes = [c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]
    lib.amgmpcg_cnn_get_gradients.argtypes = [c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]
    lib.amgmpcg_cnn_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.amgmpcg_cnn_gradients.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double)]
    lib.amgmpcg_cnn_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float,
                                           POINTER(c_double)]
    lib.amgmpcg_cnn_time_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_double)]
    lib.amgmpcg_cnn_energy_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                            ctypes.c_float, POINTER(c_double)]
    lib.amgmpcg_energy_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                        POINTER(c_double)]
    lib.amgmpcg_cnn_layer.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p]
    lib.amgmpcg_cnn_destroy.argtypes = [c_void_p]
    lib.amgmpcg_cnn_destroy.restype = None
    lib.amgmpcg_attach_cnn.argtypes = [c_void_p, c_void_p]
    lib.amgmpcg_log_kappa.argtypes = [c_void_p, c_void_p]
    lib.amgmpcg_make_pairs.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_int32, c_void_p,
                                       c_void_p]
    for name in ("amgmpcg_setup_grid", "amgmpcg_solve", "amgmpcg_solve_host", "amgmpcg_mg_block",
                 "amgmpcg_level_count", "amgmpcg_level_size", "amgmpcg_level_stencil", "amgmpcg_history",
                 "amgmpcg_residual", "amgmpcg_cnn_create", "amgmpcg_cnn_set_weights", "amgmpcg_cnn_get_weights",
                 "amgmpcg_cnn_get_gradients", "amgmpcg_cnn_forward", "amgmpcg_cnn_gradients",
                 "amgmpcg_cnn_train_step", "amgmpcg_cnn_time_forward", "amgmpcg_cnn_layer", "amgmpcg_cnn_energy_step", "amgmpcg_energy_grad", "amgmpcg_attach_cnn", "amgmpcg_log_kappa",
                 "amgmpcg_make_pairs"):
        getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def last_error() -> str:
    return load().amgmpcg_last_error().decode()


def status_string(code: int) -> str:
    return load().amgmpcg_status_string(code).decode()


def _check(code: int, allow=(OK,)):
    if code not in allow:
        raise AmgMpcgError(code, last_error() or status_string(code))
    return code


def default_options(**kw) -> Options:
    o = Options()
    load().amgmpcg_default_options(byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def gram_pinv(G: np.ndarray, tau: float):
    """Device pseudo-inverse of one Gram matrix; returns (Gplus, rank)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    nb = G.shape[0]
    out = np.empty((nb, nb))
    rank = c_int32()
    _check(load().amgmpcg_gram_pinv(G.ctypes.data_as(POINTER(c_double)), nb, float(tau),
                                    out.ctypes.data_as(POINTER(c_double)), byref(rank)))
    return out, rank.value


def gram_pinv_noalloc(G: np.ndarray, tau: float):
    """gram_pinv through the entry point that allocates no device memory."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    nb = G.shape[0]
    out = np.empty((nb, nb))
    rank = c_int32()
    _check(load().amgmpcg_gram_pinv_noalloc(G.ctypes.data_as(POINTER(c_double)), nb, float(tau),
                                            out.ctypes.data_as(POINTER(c_double)), byref(rank)))
    return out, rank.value


def _current_stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """setup(A, hierarchy) on a structured grid; solve(b, x0, tol) on device tensors."""

    def __init__(self, dim: int, n: int, nlevels: int, kappa: Optional[np.ndarray] = None,
                 stream=None, stencil: Optional[np.ndarray] = None, **options):
        lib = load()
        self._lib = lib
        self.dim, self.n, self.nlevels = dim, n, nlevels
        self.N = n ** dim
        self._kappa = None
        kp = None
        if kappa is not None:
            self._kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
            if self._kappa.size != (n + 2) ** dim:
                raise ValueError("kappa must have (n+2)^dim node values")
            kp = self._kappa.ctypes.data_as(POINTER(c_double))
        self.grid = Grid(dim, n, nlevels, kp)
        self.options = default_options(**options)
        self.stream = _current_stream() if stream is None else stream
        h = c_void_p()
        if stencil is None:
            _check(lib.amgmpcg_setup_grid(byref(self.grid), byref(self.options), self.stream, byref(h)))
        else:
            # constant 9-point finest stencil (2D), rows dy = -1, 0, 1
            self._stencil = np.ascontiguousarray(stencil, dtype=np.float64).reshape(-1)
            if self._stencil.size != 9:
                raise ValueError("stencil must have 9 entries")
            _check(lib.amgmpcg_setup_stencil(byref(self.grid), self._stencil.ctypes.data_as(POINTER(c_double)),
                                             byref(self.options), self.stream, byref(h)))
        self._h = h
        nl, nb = c_int32(), c_int32()
        _check(lib.amgmpcg_level_count(h, byref(nl), byref(nb)))
        self.nb = nb.value

    @classmethod
    def from_csr(cls, A, prolongations, restrict_scale: float = 1.0, stream=None, **options) -> "Solver":
        """setup(A, hierarchy) for a general SPD matrix A and prolongations
        P_l (level l -> l+1, coarsest first; scipy.sparse matrices), with
        R_l = restrict_scale P_l^T and Galerkin coarse operators."""
        lib = load()
        self = cls.__new__(cls)
        self._lib = lib
        self.dim, self.nlevels = 0, len(prolongations) + 1
        self.N = self.n = int(A.shape[0])
        self._kappa = None
        keep: list = []
        a = _csr_struct(A, keep)
        arr = (CsrMatrix * max(1, len(prolongations)))()
        for l, P in enumerate(prolongations):
            arr[l] = _csr_struct(P, keep)
        H = Hierarchy(self.nlevels, arr if prolongations else None, float(restrict_scale))
        self.options = default_options(**options)
        self.stream = _current_stream() if stream is None else stream
        h = c_void_p()
        _check(lib.amgmpcg_setup_csr(byref(a), byref(H), byref(self.options), self.stream, byref(h)))
        self._h = h
        nl, nb = c_int32(), c_int32()
        _check(lib.amgmpcg_level_count(h, byref(nl), byref(nb)))
        self.nb = nb.value
        return self

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.amgmpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x=None, tol: float = 1e-8, maxit: int = 0, allow=(OK, MAXIT, BREAKDOWN, NONFINITE)):
        """Solve A x = b.  b, x: float64 device tensors of n^dim entries.

        x (if given) holds x_0 and is overwritten with the result.  Returns
        (x, info dict).
        """
        import torch
        if b.dtype != torch.float64 or not b.is_cuda or not b.is_contiguous() or b.numel() != self.N:
            raise ValueError("b must be a contiguous float64 device tensor of n^dim entries")
        if x is None:
            x = torch.zeros_like(b)
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != self.N:
            raise ValueError("x must be a contiguous float64 device tensor of n^dim entries")
        info = Info()
        code = self._lib.amgmpcg_solve(self._h, c_void_p(b.data_ptr()), c_void_p(x.data_ptr()), float(tol),
                                       int(maxit), byref(info))
        _check(code, allow)
        return x, info.as_dict()

    def solve_host(self, b: np.ndarray, x0: Optional[np.ndarray] = None, tol: float = 1e-8, maxit: int = 0):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.N) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        info = Info()
        code = self._lib.amgmpcg_solve_host(self._h, b.ctypes.data_as(POINTER(c_double)),
                                            x.ctypes.data_as(POINTER(c_double)), float(tol), int(maxit),
                                            byref(info))
        _check(code, (OK, MAXIT, BREAKDOWN, NONFINITE))
        return x, info.as_dict()

    def mg_block(self, r):
        """Z = [z^0 | ... | z^L] for a float64 device residual; returns (nb, N)."""
        import torch
        Z = torch.empty((self.nb, self.N), dtype=torch.float64, device=r.device)
        _check(self._lib.amgmpcg_mg_block(self._h, c_void_p(r.data_ptr()), c_void_p(Z.data_ptr())))
        return Z

    def _vec(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.N:
            raise ValueError(f"{name} must be a contiguous float64 device tensor of n^dim entries")
        return c_void_p(t.data_ptr())

    def residual(self, b, x):
        """r = b - A x (FP64 finest operator) as a new device tensor."""
        import torch
        r = torch.empty_like(b)
        _check(self._lib.amgmpcg_residual(self._h, self._vec(b, "b"), self._vec(x, "x"), c_void_p(r.data_ptr())))
        return r

    def energy_grad(self, d, r, e, marginal: bool = False):
        """(loss, dL/dd) of the energy loss of direction d (FP64, no network)."""
        import torch
        g = torch.empty_like(d)
        loss = c_double()
        _check(self._lib.amgmpcg_energy_grad(self._h, self._vec(d, "d"), self._vec(r, "r"), self._vec(e, "e"),
                                             int(bool(marginal)), c_void_p(g.data_ptr()), byref(loss)))
        return loss.value, g

    def workspace_bytes(self) -> int:
        """Device bytes the handle's buffers take: the size of a workspace
        that amgmpcg_bind_workspace can route them through."""
        v = ctypes.c_int64()
        _check(self._lib.amgmpcg_workspace_bytes(self._h, byref(v)))
        return v.value

    def bind_workspace(self, ws=None):
        """Move the handle's device buffers into a caller-owned device
        tensor (uint8, at least workspace_bytes(), 256-byte aligned); a new
        one is allocated by torch when ws is None.  The tensor is kept alive
        with this object.  Returns it."""
        import torch
        if ws is None:
            ws = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
        _check(self._lib.amgmpcg_bind_workspace(self._h, c_void_p(ws.data_ptr()),
                                                ws.numel() * ws.element_size()))
        self._ws = ws
        return ws

    def attach(self, net: Optional["Network"]):
        """Append the network's output as one more search direction (None removes it)."""
        _check(self._lib.amgmpcg_attach_cnn(self._h, None if net is None else net._h))
        self._net = net
        nl, nb = c_int32(), c_int32()
        _check(self._lib.amgmpcg_level_count(self._h, byref(nl), byref(nb)))
        self.nb = nb.value

    def log_kappa(self):
        """The network's normalised log-kappa input channel (bfloat16 device tensor)."""
        import torch
        lk = torch.empty(self.N, dtype=torch.bfloat16, device="cuda")
        _check(self._lib.amgmpcg_log_kappa(self._h, c_void_p(lk.data_ptr())))
        return lk

    def make_pairs(self, b, xs, ks):
        """(R, E): rows r_k = b - A x_k and e_k = xs - x_k for k in ks (x_0 = 0)."""
        import torch
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        R = torch.empty((len(ks), self.N), dtype=torch.float64, device=b.device)
        E = torch.empty_like(R)
        _check(self._lib.amgmpcg_make_pairs(self._h, self._vec(b, "b"), self._vec(xs, "xs"),
                                            ks.ctypes.data_as(POINTER(c_int32)), len(ks), c_void_p(R.data_ptr()),
                                            c_void_p(E.data_ptr())))
        return R, E

    def level_size(self, level: int) -> int:
        v = c_int32()
        _check(self._lib.amgmpcg_level_size(self._h, level, byref(v)))
        return v.value

    def level_stencil(self, level: int) -> np.ndarray:
        nl = self.level_size(level)
        S = 9 if self.dim == 2 else 27
        out = np.empty(S * nl ** self.dim)
        _check(self._lib.amgmpcg_level_stencil(self._h, level, out.ctypes.data_as(POINTER(c_double))))
        return out.reshape(S, nl ** self.dim)

    KERNELS = ("update_r", "fine_smooth", "restrict_fine", "coarse_smooth", "prolong_top", "fine_W",
               "update_xP", "spmm_gram", "residual")

    def time_kernels(self, reps: int = 50) -> dict:
        """Average ms per launch of each hot kernel (HIP events, handle stream)."""
        out = np.zeros(16)
        cnt = c_int32()
        _check(self._lib.amgmpcg_time_kernels(self._h, reps, out.ctypes.data_as(POINTER(c_double)), 16,
                                              byref(cnt)))
        return {k: float(out[i]) for i, k in enumerate(self.KERNELS[: cnt.value])}

    SECTIONS = ("update_r", "fine_smooth", "restrict", "coarse_smooth", "prolong", "learned", "fine_W",
                "reduce_beta", "update_xP", "refresh", "spmm_gram", "reduce_alpha", "iteration",
                "update_xP_kernel")

    def profile_solve(self, b, x=None, tol: float = 1e-8, maxit: int = 0):
        """Solve with per-section HIP-event timing inside the iterations.

        Returns (x, info, {section: average ms per full iteration}, samples).
        The sections span consecutive stream events (launch latency included);
        "update_xP_kernel" is the x/P update's dispatch alone."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        out = np.zeros(16)
        cnt, smp = c_int32(), c_int32()
        info = Info()
        code = self._lib.amgmpcg_profile_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), float(tol), int(maxit),
                                               byref(info), out.ctypes.data_as(POINTER(c_double)), 16, byref(cnt),
                                               byref(smp))
        _check(code, (OK, MAXIT, BREAKDOWN, NONFINITE))
        return x, info.as_dict(), {k: float(out[i]) for i, k in enumerate(self.SECTIONS[: cnt.value])}, smp.value

    def history(self, cap: int = 100000) -> Tuple[np.ndarray, np.ndarray]:
        a = np.empty(cap * self.nb)
        r = np.empty(cap + 1)
        cnt = c_int32()
        _check(self._lib.amgmpcg_history(self._h, cap, a.ctypes.data_as(POINTER(c_double)),
                                         r.ctypes.data_as(POINTER(c_double)), byref(cnt)))
        k = cnt.value
        return a[: k * self.nb].reshape(k, self.nb), r[: k + 1]


class BatchedSolver:
    """Many independent Poisson problems solved together (batched launches,
    one HIP graph of k_poll iterations for all of them).

    problems: sequence of (dim, n, nlevels).  Vectors are concatenated in
    problem order (problem i starts at sum_{j<i} n_j^dim).
    """

    def __init__(self, problems, stream=None, **options):
        lib = load()
        self._lib = lib
        self.problems = [tuple(int(v) for v in p) for p in problems]
        arr = (Grid * len(self.problems))()
        for i, (d, n, nl) in enumerate(self.problems):
            arr[i] = Grid(d, n, nl, None)
        self.sizes = [n ** d for d, n, _ in self.problems]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.N = int(self.offsets[-1])
        self.options = default_options(**options)
        self.stream = _current_stream() if stream is None else stream
        h = c_void_p()
        _check(lib.amgmpcg_setup_batched(len(self.problems), arr, byref(self.options), self.stream, byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.amgmpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        """Device bytes the handle's buffers take (allocated at setup)."""
        v = ctypes.c_int64()
        _check(self._lib.amgmpcg_workspace_bytes(self._h, byref(v)))
        return v.value

    def solve(self, b, x=None, tol: float = 1e-8, maxit: int = 0):
        """b, x: contiguous float64 device tensors of all problems concatenated.

        Returns (x, list of per-problem info dicts, device ms of the launch).
        """
        import torch
        if b.dtype != torch.float64 or not b.is_cuda or not b.is_contiguous() or b.numel() != self.N:
            raise ValueError("b must be a contiguous float64 device tensor of all problems")
        if x is None:
            x = torch.zeros_like(b)
        if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != self.N:
            raise ValueError("x must match b")
        infos = (Info * len(self.problems))()
        ms = c_double()
        code = self._lib.amgmpcg_solve_batched(self._h, c_void_p(b.data_ptr()), c_void_p(x.data_ptr()),
                                               float(tol), int(maxit), infos, byref(ms))
        _check(code, (OK, MAXIT, BREAKDOWN, NONFINITE))
        return x, [i.as_dict() for i in infos], ms.value


def cnn_weight_count() -> int:
    return int(load().amgmpcg_cnn_weight_count())


# Layer shapes (taps, Cin, Cout) in weight-array order.
CNN_LAYERS = (("w1", 27, 16, 16), ("w2", 27, 16, 16), ("w3", 27, 16, 32), ("w4", 27, 32, 32),
              ("w5", 27, 32, 64), ("w6", 27, 64, 64), ("w7", 27, 96, 32), ("w8", 27, 32, 32),
              ("w9", 27, 48, 16), ("w10", 27, 16, 16), ("w11", 1, 16, 16))


class Network:
    """The U-Net learned direction for n^3 grids (device weights, Adam state)."""

    def __init__(self, n: int, seed: int = 0, stream=None):
        lib = load()
        self._lib = lib
        self.n = n
        self.N = n ** 3
        self.stream = _current_stream() if stream is None else stream
        h = c_void_p()
        _check(lib.amgmpcg_cnn_create(int(n), int(seed), self.stream, byref(h)))
        self._h = h
        self.count = cnn_weight_count()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.amgmpcg_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.N:
            raise ValueError(f"{name} must be a contiguous float64 device tensor of n^3 entries")
        return c_void_p(t.data_ptr())

    def _lk(self, lk):
        import torch
        if lk is None:
            return None
        if lk.dtype != torch.bfloat16 or not lk.is_cuda or not lk.is_contiguous() or lk.numel() != self.N:
            raise ValueError("lk must be a contiguous bfloat16 device tensor of n^3 entries")
        return c_void_p(lk.data_ptr())

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.count, dtype=np.float32)
        _check(self._lib.amgmpcg_cnn_get_weights(self._h, w.ctypes.data_as(POINTER(ctypes.c_float)), self.count))
        return w

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        _check(self._lib.amgmpcg_cnn_set_weights(self._h, w.ctypes.data_as(POINTER(ctypes.c_float)), w.size))

    def get_gradients(self) -> np.ndarray:
        g = np.empty(self.count, dtype=np.float32)
        _check(self._lib.amgmpcg_cnn_get_gradients(self._h, g.ctypes.data_as(POINTER(ctypes.c_float)), self.count))
        return g

    @staticmethod
    def split(flat: np.ndarray) -> dict:
        """Flat weight array -> {name: (taps, Cout, Cin) array} (w11: (Cout, Cin))."""
        out, off = {}, 0
        for name, taps, cin, cout in CNN_LAYERS:
            cnt = taps * cin * cout
            a = np.asarray(flat[off:off + cnt]).reshape(taps, cout, cin)
            out[name] = a[0] if taps == 1 else a
            off += cnt
        return out

    @staticmethod
    def join(layers: dict) -> np.ndarray:
        return np.concatenate([np.asarray(layers[name], dtype=np.float32).reshape(-1)
                               for name, *_ in CNN_LAYERS])

    def forward(self, r, lk=None, allow=(OK, NONFINITE)):
        """d = N(r) as a new float64 device tensor; returns (d, status)."""
        import torch
        d = torch.empty_like(r)
        code = self._lib.amgmpcg_cnn_forward(self._h, self._vec(r, "r"), self._lk(lk), c_void_p(d.data_ptr()))
        _check(code, allow)
        return d, code

    def gradients(self, r, e, lk=None) -> float:
        loss = c_double()
        _check(self._lib.amgmpcg_cnn_gradients(self._h, self._vec(r, "r"), self._lk(lk), self._vec(e, "e"),
                                               byref(loss)))
        return loss.value

    def train_step(self, r, e, lr: float, lk=None) -> float:
        loss = c_double()
        _check(self._lib.amgmpcg_cnn_train_step(self._h, self._vec(r, "r"), self._lk(lk), self._vec(e, "e"),
                                                float(lr), byref(loss)))
        return loss.value

    def energy_step(self, solver: "Solver", r, e, lr: float = 0.0, lk=None, marginal: bool = False) -> float:
        """Energy-loss step with the finest operator of `solver` (lr = 0: gradients only);
        marginal: the loss on top of the solver's level-correction block of r."""
        loss = c_double()
        _check(self._lib.amgmpcg_cnn_energy_step(self._h, solver._h, self._vec(r, "r"), self._lk(lk),
                                                 self._vec(e, "e"), int(bool(marginal)), float(lr), byref(loss)))
        return loss.value

    def layer(self, layer: int, op: int, A, B=None):
        """One layer on bfloat16 device tensors of shape (S, S, S, C): op 0
        forward (+ReLU; the output layer gives FP32 channel 0 only), op 1 data
        gradient, op 2 weight gradient (A = output gradient, B = layer
        input).  Returns a new device tensor."""
        import torch
        _, taps, cin, cout = CNN_LAYERS[layer]
        S = A.shape[0]
        for t in (A, B):
            if t is not None and (t.dtype != torch.bfloat16 or not t.is_cuda or not t.is_contiguous()
                                  or t.dim() != 4 or t.shape[:3] != (S, S, S)):
                raise ValueError("tensors must be contiguous bfloat16 (S, S, S, C) device tensors")
        need_a = cin if op == 0 else cout
        if A.shape[3] != need_a or (op == 2 and (B is None or B.shape[3] != cin)):
            raise ValueError("channel count does not match the layer")
        if op == 0 and layer == 10:
            out = torch.empty((S, S, S, 1), dtype=torch.float32, device=A.device)
        elif op == 0:
            out = torch.empty((S, S, S, cout), dtype=torch.bfloat16, device=A.device)
        elif op == 1:
            out = torch.empty((S, S, S, cin), dtype=torch.bfloat16, device=A.device)
        else:
            out = torch.empty((taps, cout, cin), dtype=torch.float32, device=A.device)
        _check(self._lib.amgmpcg_cnn_layer(self._h, layer, op, S, c_void_p(A.data_ptr()),
                                           None if B is None else c_void_p(B.data_ptr()),
                                           c_void_p(out.data_ptr())))
        return out

    def time_forward(self, r, lk=None, reps: int = 10) -> float:
        ms = c_double()
        _check(self._lib.amgmpcg_cnn_time_forward(self._h, self._vec(r, "r"), self._lk(lk), int(reps), byref(ms)))
        return ms.value
