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
INVALID_ARG, NOT_SPD, DIM_MISMATCH, NONFINITE, OOM, HIP_ERROR, UNAVAILABLE = -1, -2, -3, -4, -5, -6, -7


class Grid(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n", c_int32), ("nlevels", c_int32), ("kappa", POINTER(c_double))]


class Options(ctypes.Structure):
    _fields_ = [("m", c_int32), ("nu", c_int32), ("omega", c_double), ("maxit", c_int32),
                ("precision", c_int32), ("pinv_tau", c_double), ("k_poll", c_int32),
                ("record_history", c_int32), ("refresh_drop", c_double)]


class Info(ctypes.Structure):
    _fields_ = [("status", c_int32), ("iterations", c_int32), ("bnorm", c_double), ("relres", c_double),
                ("refreshes", c_int32), ("nb", c_int32), ("solve_ms", c_double)]

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
    lib = ctypes.CDLL(path)
    lib.amgmpcg_default_options.argtypes = [POINTER(Options)]
    lib.amgmpcg_default_options.restype = None
    lib.amgmpcg_setup_grid.argtypes = [POINTER(Grid), POINTER(Options), c_void_p, POINTER(c_void_p)]
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
    lib.amgmpcg_setup_batched.argtypes = [c_int32, POINTER(Grid), POINTER(Options), c_void_p, POINTER(c_void_p)]
    lib.amgmpcg_setup_batched.restype = c_int32
    lib.amgmpcg_solve_batched.argtypes = [c_void_p, c_void_p, c_void_p, c_double, c_int32, POINTER(Info),
                                          POINTER(c_double)]
    lib.amgmpcg_solve_batched.restype = c_int32
    lib.amgmpcg_batched_size.argtypes = [c_void_p, POINTER(c_int32), POINTER(ctypes.c_int64)]
    lib.amgmpcg_batched_size.restype = c_int32
    lib.amgmpcg_gram_pinv.argtypes = [POINTER(c_double), c_int32, c_double, POINTER(c_double), POINTER(c_int32)]
    lib.amgmpcg_gram_pinv.restype = c_int32
    lib.amgmpcg_destroy.argtypes = [c_void_p]
    lib.amgmpcg_destroy.restype = None
    lib.amgmpcg_status_string.argtypes = [c_int32]
    lib.amgmpcg_status_string.restype = ctypes.c_char_p
    lib.amgmpcg_last_error.argtypes = []
    lib.amgmpcg_last_error.restype = ctypes.c_char_p
    for name in ("amgmpcg_setup_grid", "amgmpcg_solve", "amgmpcg_solve_host", "amgmpcg_mg_block",
                 "amgmpcg_level_count", "amgmpcg_level_size", "amgmpcg_level_stencil", "amgmpcg_history"):
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


def _current_stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """setup(A, hierarchy) on a structured grid; solve(b, x0, tol) on device tensors."""

    def __init__(self, dim: int, n: int, nlevels: int, kappa: Optional[np.ndarray] = None,
                 stream=None, **options):
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
        _check(lib.amgmpcg_setup_grid(byref(self.grid), byref(self.options), self.stream, byref(h)))
        self._h = h
        nl, nb = c_int32(), c_int32()
        _check(lib.amgmpcg_level_count(h, byref(nl), byref(nb)))
        self.nb = nb.value

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

    def history(self, cap: int = 100000) -> Tuple[np.ndarray, np.ndarray]:
        a = np.empty(cap * self.nb)
        r = np.empty(cap + 1)
        cnt = c_int32()
        _check(self._lib.amgmpcg_history(self._h, cap, a.ctypes.data_as(POINTER(c_double)),
                                         r.ctypes.data_as(POINTER(c_double)), byref(cnt)))
        k = cnt.value
        return a[: k * self.nb].reshape(k, self.nb), r[: k + 1]


class BatchedSolver:
    """Many independent Poisson problems solved by one persistent launch.

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
