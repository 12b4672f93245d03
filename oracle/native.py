"""Loader for the oracle's C helpers (test infrastructure only).

grad_ld.c is plain C with OpenMP, compiled with gcc into
oracle/_build/libtikoracle.so by ``build_native`` (the package build calls
it).  It shares nothing with the GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "grad_ld.c")
LIB = os.path.join(HERE, "_build", "libtikoracle.so")
_lib: Optional[ctypes.CDLL] = None


def build_native() -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC], check=True)
    os.replace(tmp, LIB)
    return LIB


def lib() -> Optional[ctypes.CDLL]:
    """The compiled helper, or None when it has not been built."""
    global _lib
    if _lib is None and os.path.exists(LIB):
        L = ctypes.CDLL(LIB)
        L.oracle_tik_gradient.restype = ctypes.c_int
        L.oracle_tik_gradient.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        _lib = L
    return _lib


def gradient_ld(A: np.ndarray, b: np.ndarray, lams: np.ndarray, X: np.ndarray) -> Optional[np.ndarray]:
    """A^T (b - A X) - X diag(lams) accumulated in long double, or None without the helper."""
    L = lib()
    if L is None:
        return None
    A = np.asarray(A)
    if A.dtype not in (np.float32, np.float64):
        A = A.astype(np.float64)
    if not A.flags.f_contiguous:
        A = np.asfortranarray(A)
    m, n = A.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    lams = np.ascontiguousarray(lams, dtype=np.float64)
    X = np.asfortranarray(np.asarray(X, dtype=np.float64).reshape(n, -1))
    N = X.shape[1]
    G = np.empty((n, N), dtype=np.float64, order="F")
    rc = L.oracle_tik_gradient(A.ctypes.data, 1 if A.dtype == np.float32 else 0, m, n, m,
                               b.ctypes.data, X.ctypes.data, lams.ctypes.data, N, G.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_tik_gradient failed ({rc})")
    return G
