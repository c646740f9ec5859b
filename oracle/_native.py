"""Loader for the oracle's plain-C exact dot product (``exactdot.c``).

The shared object is compiled with gcc next to its source the first time it
is needed (or by ``build()``), and loaded with ctypes.  It is test
infrastructure and is never linked into the HIP library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exactdot.c")
_LIB = os.path.join(_HERE, "libexactdot.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile exactdot.c with gcc (OpenMP over matrix rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-std=gnu11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            L.exact_dot.restype = ctypes.c_double
            L.exact_dot.argtypes = [dp, ctypes.c_long, dp, ctypes.c_long, ctypes.c_long]
            L.exact_matvec.restype = None
            L.exact_matvec.argtypes = [dp, ctypes.c_long, ctypes.c_long, ctypes.c_long, dp, dp]
            L.exact_matvec_reference.restype = None
            L.exact_matvec_reference.argtypes = L.exact_matvec.argtypes
            L.exact_fallbacks.restype = ctypes.c_long
            L.exact_fallbacks.argtypes = []
            L.exact_sum.restype = ctypes.c_double
            L.exact_sum.argtypes = [dp, ctypes.c_long]
            L.exact_threads.restype = ctypes.c_int
            L.exact_threads.argtypes = []
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def exact_dot(x, y) -> float:
    """Nearest double to the exact sum of x[i] * y[i]."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    if x.shape != y.shape:
        raise ValueError("length mismatch")
    return float(lib().exact_dot(_ptr(x), 1, _ptr(y), 1, x.size))


def exact_matvec(a, x) -> np.ndarray:
    """Row-wise correctly rounded product A @ x (A two-dimensional).

    Each row is decided by a certified error-free-transformation enclosure
    where that settles the rounding, and by the exact superaccumulator
    otherwise; either way the entry is the nearest double to the exact sum.
    """
    a = np.ascontiguousarray(a, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    rows, cols = a.shape
    if cols != x.size:
        raise ValueError("shape mismatch")
    out = np.empty(rows)
    lib().exact_matvec(_ptr(a), rows, cols, cols, _ptr(x), _ptr(out))
    return out


def exact_matvec_reference(a, x) -> np.ndarray:
    """The same product by the superaccumulator alone, row by row."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    rows, cols = a.shape
    if cols != x.size:
        raise ValueError("shape mismatch")
    out = np.empty(rows)
    lib().exact_matvec_reference(_ptr(a), rows, cols, cols, _ptr(x), _ptr(out))
    return out


def exact_fallbacks() -> int:
    """Rows exact_matvec has handed to the superaccumulator so far."""
    return int(lib().exact_fallbacks())


def exact_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return float(lib().exact_sum(_ptr(x), x.size))


def exact_threads() -> int:
    """Threads the row-parallel exact matrix-vector product uses."""
    return int(lib().exact_threads())
