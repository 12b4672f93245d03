"""Thin ctypes binding of libtik (include/tik.h): argument marshalling only.

Every step of the method runs in the HIP library; this module only turns
torch device tensors into the C structs and pointers the ABI takes, and
allocates the device workspaces the library asks for (torch owns all device
memory).  If libtik.so is missing the import of any entry point raises:
there is no fallback path.

Layout: a column-major m x n matrix is a contiguous torch tensor of shape
(n, m) (its transpose in row-major terms); `colmajor()` converts.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtik.so")

# enums (include/tik.h)
OK, EINVAL, EWORKSPACE, EHIP, ENOTSUP = 0, -1, -2, -3, -4
ST_CONVERGED, ST_MAXIT, ST_NOTPD, ST_IR_STALL, ST_NONFINITE, ST_QR = 0, 1, 2, 3, 4, 5
F64, F32, BF16, F16 = 0, 1, 2, 3
SRHT, GAUSS, SPARSE = 0, 1, 2
ROUTE_CHOL, ROUTE_LOWRANK = 0, 1
PLAIN_F64_PER_LAMBDA, F64_BATCHED, MIXED_BATCHED = 0, 1, 2

EXPORTS = [
    "tik_sketch_bytes", "tik_sketch", "tik_sketch_data", "tik_precond_bytes", "tik_precond",
    "tik_precond_data", "tik_precond_sigma",
    "tik_lsqr_batch_bytes", "tik_lsqr_batch", "tik_sketch_free", "tik_precond_free",
    "tik_last_error", "tik_version", "tik_prof_enable", "tik_prof_reset", "tik_prof_query",
    "tik_lsqr_info", "tik_set_option", "tik_get_option", "tik_lsqr_batch_static",
    "tik_lcurve_bytes", "tik_lcurve", "tik_lcurve_corner",
    "tik_tune_bytes", "tik_tune", "tik_tune_save", "tik_tune_load", "tik_last_tiles",
    "tik_precond_sweeps", "tik_lsqr_times",
]


class TikError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"libtik error {rc}: {msg}")
        self.rc = rc


class CProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("a_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("A", ctypes.c_void_p), ("b", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtik.so (built in-tree by build.py); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_07329_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_size_t, ctypes.c_double, ctypes.c_uint64)
    P = ctypes.POINTER
    L.tik_sketch_bytes.argtypes = [P(CProblem), i32, i32, i32, P(i64), P(sz)]
    L.tik_sketch.argtypes = [P(CProblem), i32, i32, i32, P(i64), u64, vp, sz, vp, P(vp)]
    L.tik_sketch_data.argtypes = [vp, i32, P(vp), P(i64), P(i64)]
    L.tik_precond_bytes.argtypes = [vp, i32, i32, P(sz)]
    L.tik_precond.argtypes = [vp, i32, P(dbl), i32, dbl, vp, sz, vp, P(vp), P(dbl), P(i32)]
    L.tik_precond_data.argtypes = [vp, i32, i32, P(vp), P(i64), P(i64)]
    L.tik_precond_sigma.argtypes = [vp, i32, P(vp), P(i64)]
    L.tik_lsqr_batch_bytes.argtypes = [P(CProblem), i32, vp, i32, P(sz)]
    L.tik_lsqr_batch.argtypes = [P(CProblem), i32, vp, i32, dbl, i32, P(vp), vp, vp, vp, vp, sz, vp]
    L.tik_sketch_free.argtypes = [vp]
    L.tik_sketch_free.restype = None
    L.tik_precond_free.argtypes = [vp]
    L.tik_precond_free.restype = None
    L.tik_last_error.restype = ctypes.c_char_p
    L.tik_prof_enable.argtypes = [i32]
    L.tik_prof_query.argtypes = [ctypes.c_char_p, P(dbl), P(i64)]
    L.tik_lsqr_info.argtypes = [P(i32), P(i32)]
    L.tik_set_option.argtypes = [ctypes.c_char_p, i64]
    L.tik_lcurve_bytes.argtypes = [P(CProblem), i32, P(sz)]
    L.tik_lcurve.argtypes = [P(CProblem), i32, i32, P(vp), vp, vp, vp, sz, vp]
    L.tik_lcurve_corner.argtypes = [P(dbl), P(dbl), P(dbl), i32, P(i32), P(dbl)]
    L.tik_tune_bytes.argtypes = [P(CProblem), i32, vp, P(sz)]
    L.tik_precond_sweeps.argtypes = [vp, i32, P(i32)]
    L.tik_lsqr_times.argtypes = [P(dbl), i64]
    L.tik_tune.argtypes = [P(CProblem), i32, vp, i32, vp, sz, vp, P(i32), P(dbl), P(dbl)]
    L.tik_tune_save.argtypes = [ctypes.c_char_p]
    L.tik_tune_load.argtypes = [ctypes.c_char_p, P(i32)]
    L.tik_last_tiles.argtypes = [ctypes.c_char_p, i32]
    L.tik_lsqr_batch_static.argtypes = [P(CProblem), i32, vp, i32, dbl, i32, P(vp), vp, vp, vp, vp]
    L.tik_get_option.argtypes = [ctypes.c_char_p, P(i64)]
    for name in ("tik_sketch_bytes", "tik_sketch", "tik_sketch_data", "tik_precond_bytes",
                 "tik_precond", "tik_precond_data", "tik_lsqr_batch_bytes", "tik_lsqr_batch", "tik_version",
                 "tik_prof_enable", "tik_prof_reset", "tik_prof_query", "tik_lsqr_info",
                 "tik_set_option", "tik_get_option", "tik_lsqr_batch_static",
                 "tik_lcurve_bytes", "tik_lcurve", "tik_lcurve_corner", "tik_tune_bytes", "tik_tune",
                 "tik_tune_save", "tik_tune_load", "tik_last_tiles", "tik_precond_sweeps", "tik_lsqr_times"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != OK:
        raise TikError(rc, lib().tik_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


def colmajor(a: np.ndarray, device="cuda") -> torch.Tensor:
    """Column-major device copy of an (m, n) numpy matrix: a (n, m) tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(device)


@dataclass
class Problems:
    """Device problems: At[k] is (n_k, m_k) (column-major A_k), b[k] is (m_k,) float64."""

    At: List[torch.Tensor]
    b: List[torch.Tensor]
    c: ctypes.Array = field(init=False)

    def __post_init__(self):
        arr = (CProblem * len(self.At))()
        for k, (At, b) in enumerate(zip(self.At, self.b)):
            if At.dim() != 2 or not At.is_contiguous() or not At.is_cuda:
                raise ValueError("At must be a contiguous 2-D device tensor (column-major A)")
            if At.dtype not in (torch.float64, torch.float32):
                raise ValueError("A must be float64 or float32")
            if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != At.shape[1]:
                raise ValueError("b must be a contiguous float64 vector of length m")
            n, m = At.shape
            arr[k] = CProblem(m, n, m, F64 if At.dtype == torch.float64 else F32, 0,
                              At.data_ptr(), b.data_ptr())
        self.c = arr

    @property
    def count(self) -> int:
        return len(self.At)

    def shape(self, k: int):
        return int(self.At[k].shape[1]), int(self.At[k].shape[0])

    @staticmethod
    def from_numpy(As: Sequence[np.ndarray], bs: Sequence[np.ndarray], device="cuda") -> "Problems":
        return Problems([colmajor(A, device) for A in As],
                        [torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).to(device) for b in bs])


@dataclass
class Sketch:
    handle: ctypes.c_void_p
    ws: torch.Tensor
    probs: Problems

    def Y(self, k: int = 0) -> np.ndarray:
        """Problem k's sketch as stored (tall: Y, s x n; wide: Y^T, s x m), on the host."""
        ptr, r, c = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tik_sketch_data(self.handle, k, ctypes.byref(ptr), ctypes.byref(r), ctypes.byref(c)))
        base = self.ws.data_ptr()
        off = ptr.value - base
        nbytes = r.value * c.value * 8
        host = self.ws[off:off + nbytes].cpu().numpy().view(np.float64)
        return host.reshape(c.value, r.value).T.copy()

    def __del__(self):
        if _lib is not None and self.handle:
            _lib.tik_sketch_free(self.handle)
            self.handle = None


@dataclass
class Precond:
    handle: ctypes.c_void_p
    ws: torch.Tensor
    sketch: Sketch
    status: np.ndarray
    sd_hat: np.ndarray
    N: int

    def data(self, k: int = 0, i: int = 0) -> np.ndarray:
        """Host copy of problem k, lambda i: R^{-1} (Cholesky route) or V[:, :s_i] (low rank)."""
        ptr, d, r = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tik_precond_data(self.handle, k, i, ctypes.byref(ptr), ctypes.byref(d),
                                      ctypes.byref(r)))
        off = ptr.value - self.ws.data_ptr()
        cols = d.value if r.value == d.value else r.value
        nbytes = d.value * cols * 8
        host = self.ws[off:off + nbytes].cpu().numpy().view(np.float64)
        return host.reshape(cols, d.value).T.copy()

    def rank(self, k: int = 0, i: int = 0) -> int:
        """Columns of the preconditioner's factor for problem k, lambda i (s_i on the low-rank route)."""
        ptr, d, r = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().tik_precond_data(self.handle, k, i, ctypes.byref(ptr), ctypes.byref(d),
                                      ctypes.byref(r)))
        return int(r.value)

    def sweeps(self, k: int = 0) -> int:
        """Jacobi sweeps of problem k's SVD (low-rank route)."""
        n = ctypes.c_int32()
        _check(lib().tik_precond_sweeps(self.handle, k, ctypes.byref(n)))
        return int(n.value)

    def sigma(self, k: int = 0) -> np.ndarray:
        """Singular values of problem k's sketch, decreasing (low-rank route)."""
        ptr, c = ctypes.c_void_p(), ctypes.c_int64()
        _check(lib().tik_precond_sigma(self.handle, k, ctypes.byref(ptr), ctypes.byref(c)))
        off = ptr.value - self.ws.data_ptr()
        return self.ws[off:off + 8 * c.value].cpu().numpy().view(np.float64).copy()

    def __del__(self):
        if _lib is not None and self.handle:
            _lib.tik_precond_free(self.handle)
            self.handle = None


def sketch(probs: Problems, embed: int, s: Sequence[int], seed: int = 0,
           sketch_dtype: int = F64, stream=None) -> Sketch:
    L = lib()
    sarr = (ctypes.c_int64 * probs.count)(*[int(v) for v in s])
    nb = ctypes.c_size_t()
    _check(L.tik_sketch_bytes(probs.c, probs.count, embed, sketch_dtype, sarr, ctypes.byref(nb)))
    ws = _workspace(nb.value, probs.At[0].device)
    h = ctypes.c_void_p()
    _check(L.tik_sketch(probs.c, probs.count, embed, sketch_dtype, sarr, ctypes.c_uint64(seed),
                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream), ctypes.byref(h)))
    return Sketch(h, ws, probs)


def precond(sk: Sketch, lambdas: np.ndarray, route: int = ROUTE_CHOL, alpha: float = 2.0,
            stream=None) -> Precond:
    L = lib()
    lams = np.ascontiguousarray(np.atleast_2d(np.asarray(lambdas, dtype=np.float64)))
    if lams.shape[0] == 1 and sk.probs.count > 1:
        lams = np.ascontiguousarray(np.repeat(lams, sk.probs.count, axis=0))
    nprob, N = lams.shape
    nb = ctypes.c_size_t()
    _check(L.tik_precond_bytes(sk.handle, route, N, ctypes.byref(nb)))
    ws = _workspace(nb.value, sk.ws.device)
    h = ctypes.c_void_p()
    sd = np.empty((nprob, N))
    st = np.empty((nprob, N), dtype=np.int32)
    _check(L.tik_precond(sk.handle, route, lams.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), N,
                         float(alpha), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                         ctypes.byref(h), sd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return Precond(h, ws, sk, st, sd, N)


@dataclass
class Result:
    X: List[torch.Tensor]       # per problem (N, n) device tensor: row i is x_{lam_i}
    iters: torch.Tensor         # (nprob, N) int32, device
    status: torch.Tensor
    relres: torch.Tensor

    def x_numpy(self, k: int = 0) -> np.ndarray:
        """Problem k's solutions as an (n, N) host array."""
        return self.X[k].cpu().numpy().T.copy()


class Solver:
    """Reusable tik_lsqr_batch call: workspace and outputs allocated once."""

    def __init__(self, probs: Problems, pc: Precond, mode: int):
        L = lib()
        self.probs, self.pc, self.mode = probs, pc, mode
        nb = ctypes.c_size_t()
        _check(L.tik_lsqr_batch_bytes(probs.c, probs.count, pc.handle, mode, ctypes.byref(nb)))
        dev = probs.At[0].device
        self.ws = _workspace(nb.value, dev)
        N = pc.N
        self.X = [torch.zeros((N, probs.shape(k)[1]), dtype=torch.float64, device=dev)
                  for k in range(probs.count)]
        self.iters = torch.zeros((probs.count, N), dtype=torch.int32, device=dev)
        self.status = torch.zeros((probs.count, N), dtype=torch.int32, device=dev)
        self.relres = torch.zeros((probs.count, N), dtype=torch.float64, device=dev)
        self._xp = (ctypes.c_void_p * probs.count)(*[x.data_ptr() for x in self.X])

    def __call__(self, tol: float, maxit: int, stream=None) -> Result:
        _check(lib().tik_lsqr_batch(self.probs.c, self.probs.count, self.pc.handle, self.mode,
                                    float(tol), int(maxit), self._xp,
                                    ctypes.c_void_p(self.iters.data_ptr()),
                                    ctypes.c_void_p(self.status.data_ptr()),
                                    ctypes.c_void_p(self.relres.data_ptr()),
                                    ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                    _stream(stream)))
        return Result(self.X, self.iters, self.status, self.relres)


def lsqr_batch(probs: Problems, pc: Precond, mode: int, tol: float, maxit: int,
               stream=None) -> Result:
    return Solver(probs, pc, mode)(tol, maxit, stream)


def lsqr_batch_static(probs: Problems, pc: Precond, mode: int, tol: float, maxit: int,
                      stream=None) -> Result:
    """tik_lsqr_batch_static: the library's static workspace, nothing allocated by the call
    (the outputs are allocated here, by the caller)."""
    dev = probs.At[0].device
    N = pc.N
    X = [torch.zeros((N, probs.shape(k)[1]), dtype=torch.float64, device=dev)
         for k in range(probs.count)]
    iters = torch.zeros((probs.count, N), dtype=torch.int32, device=dev)
    status = torch.zeros((probs.count, N), dtype=torch.int32, device=dev)
    relres = torch.zeros((probs.count, N), dtype=torch.float64, device=dev)
    xp = (ctypes.c_void_p * probs.count)(*[x.data_ptr() for x in X])
    _check(lib().tik_lsqr_batch_static(probs.c, probs.count, pc.handle, mode, float(tol), int(maxit),
                                       xp, ctypes.c_void_p(iters.data_ptr()),
                                       ctypes.c_void_p(status.data_ptr()),
                                       ctypes.c_void_p(relres.data_ptr()), _stream(stream)))
    return Result(X, iters, status, relres)


def solve(probs: Problems, lambdas, embed: int = SRHT, s: Optional[Sequence[int]] = None,
          route: int = ROUTE_CHOL, mode: int = F64_BATCHED, tol: float = 1e-10,
          maxit: int = 200, seed: int = 0, sketch_dtype: int = F64, alpha: float = 2.0):
    """Sketch, precondition and solve in one call; returns (Result, Precond)."""
    if s is None:
        s = [4 * min(probs.shape(k)) for k in range(probs.count)]
    sk = sketch(probs, embed, s, seed, sketch_dtype)
    pc = precond(sk, lambdas, route, alpha)
    return lsqr_batch(probs, pc, mode, tol, maxit), pc


def lcurve(probs: Problems, X: Sequence[torch.Tensor], stream=None):
    """tik_lcurve: (xnorm, rnorm) device tensors (nprob, N) of the solutions X[k]
    ((N, n_k) tensors as Result.X holds them: column-major n_k x N)."""
    L = lib()
    N = int(X[0].shape[0])
    nb = ctypes.c_size_t()
    _check(L.tik_lcurve_bytes(probs.c, probs.count, ctypes.byref(nb)))
    dev = X[0].device
    ws = _workspace(nb.value, dev)
    xn = torch.zeros((probs.count, N), dtype=torch.float64, device=dev)
    rn = torch.zeros((probs.count, N), dtype=torch.float64, device=dev)
    xp = (ctypes.c_void_p * probs.count)(*[x.data_ptr() for x in X])
    _check(L.tik_lcurve(probs.c, probs.count, N, xp, ctypes.c_void_p(xn.data_ptr()),
                        ctypes.c_void_p(rn.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                        _stream(stream)))
    return xn, rn


def lcurve_corner(lambdas, xnorm, rnorm):
    """tik_lcurve_corner on host arrays: (corner index, curvature array)."""
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    xn = np.ascontiguousarray(xnorm, dtype=np.float64)
    rn = np.ascontiguousarray(rnorm, dtype=np.float64)
    n = lam.size
    curv = np.empty(n, dtype=np.float64)
    c = ctypes.c_int32()
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib().tik_lcurve_corner(lam.ctypes.data_as(P), xn.ctypes.data_as(P), rn.ctypes.data_as(P),
                                   n, ctypes.byref(c), curv.ctypes.data_as(P)))
    return c.value, curv


def tune(probs: Problems, pc: Precond, iters: int = 10, stream=None):
    """tik_tune: time the candidate launch shapes on these problems, keep the fastest.
    Returns ((rows, cols, blocks), best_ms, default_ms)."""
    L = lib()
    nb = ctypes.c_size_t()
    _check(L.tik_tune_bytes(probs.c, probs.count, pc.handle, ctypes.byref(nb)))
    ws = _workspace(nb.value, probs.At[0].device)
    best = (ctypes.c_int32 * 3)()
    bms, dms = ctypes.c_double(), ctypes.c_double()
    _check(L.tik_tune(probs.c, probs.count, pc.handle, int(iters), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                      _stream(stream), best, ctypes.byref(bms), ctypes.byref(dms)))
    return (best[0], best[1], best[2]), bms.value, dms.value


def tune_save(path: str) -> None:
    _check(lib().tik_tune_save(path.encode()))


def tune_load(path: str) -> int:
    n = ctypes.c_int32()
    _check(lib().tik_tune_load(path.encode(), ctypes.byref(n)))
    return n.value


def last_tiles() -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().tik_last_tiles(buf, 512))
    return buf.value.decode()


def lsqr_times(nprob: int, N: int) -> np.ndarray:
    """tik_lsqr_times: (nprob, N) ms from the start of the last call's first solve loop to
    each solve's stop (NaN where not timed); needs set_option("record_times", 1)."""
    out = np.empty(nprob * N, dtype=np.float64)
    _check(lib().tik_lsqr_times(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nprob * N))
    return out.reshape(nprob, N)


def lsqr_info():
    """(lambdas refined with FP32 products, lambdas solved with FP64 products) of the last call."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tik_lsqr_info(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def set_option(name: str, value: int) -> None:
    _check(lib().tik_set_option(name.encode(), int(value)))


def get_option(name: str) -> int:
    v = ctypes.c_int64()
    _check(lib().tik_get_option(name.encode(), ctypes.byref(v)))
    return v.value


# ------------------------------------------------------------- profiling ---
def prof_enable(on: bool = True) -> None:
    _check(lib().tik_prof_enable(1 if on else 0))


def prof_reset() -> None:
    _check(lib().tik_prof_reset())


def prof_query(family: str):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().tik_prof_query(family.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value
