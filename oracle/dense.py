"""ctypes wrapper for the oracle's plain-C dense linear algebra (dense.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Builds oracle/_dense.so
with gcc on first use if it is not there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dense.c")
_LIB = os.path.join(_HERE, "_dense.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def build() -> str:
    """Compile dense.c (FP64, no fast-math, OpenMP) into _dense.so."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-std=c11", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_gram.argtypes = [_D, _I64, _I64, _I64, _D, _I64]
    lib.oracle_gram.restype = ctypes.c_int
    lib.oracle_gram_entries.argtypes = [_D, _I64, _I64, ctypes.POINTER(_I64),
                                        ctypes.POINTER(_I64), _I64, _D]
    lib.oracle_gradient.argtypes = [_D, _I64, _I64, _I64, _D, _D]
    lib.oracle_cholesky.argtypes = [_D, _I64, _I64]
    lib.oracle_cholesky.restype = _I64
    lib.oracle_solve_lower.argtypes = [_D, _I64, _I64, _D]
    lib.oracle_solve_lower_t.argtypes = [_D, _I64, _I64, _D]
    lib.oracle_symv_lower.argtypes = [_D, _I64, _I64, _D, _D]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the later parallel loops of the C part."""
    _load().oracle_set_num_threads(int(n))


def gram(J: np.ndarray) -> np.ndarray:
    """G = J^T J, every entry a compensated (Dot2) dot product."""
    J = _c(J)
    m, p = J.shape
    G = np.empty((p, p))
    if _load().oracle_gram(_p(J), m, p, p, _p(G), p) != 0:
        raise MemoryError("oracle_gram")
    return G


def gram_entries(J: np.ndarray, rows, cols) -> np.ndarray:
    J = _c(J)
    m, p = J.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.size)
    _load().oracle_gram_entries(_p(J), m, p, rows.ctypes.data_as(ctypes.POINTER(_I64)),
                                cols.ctypes.data_as(ctypes.POINTER(_I64)), rows.size, _p(out))
    return out


def gradient(J: np.ndarray, r: np.ndarray) -> np.ndarray:
    """g = J^T r with compensated dot products."""
    J = _c(J)
    r = _c(r)
    m, p = J.shape
    g = np.empty(p)
    _load().oracle_gradient(_p(J), m, p, p, _p(r), _p(g))
    return g


def cholesky(A: np.ndarray):
    """Lower Cholesky factor of the lower triangle of A; returns (L, info).

    info = 0 on success, else the 1-based index of the first non-positive
    pivot (LAPACK potrf convention).
    """
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    info = int(_load().oracle_cholesky(_p(L), n, n))
    return np.tril(L), info


def solve_lower(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    L = _c(L)
    x = np.array(b, dtype=np.float64, copy=True)
    _load().oracle_solve_lower(_p(L), L.shape[0], L.shape[1], _p(x))
    return x


def solve_lower_t(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    L = _c(L)
    x = np.array(b, dtype=np.float64, copy=True)
    _load().oracle_solve_lower_t(_p(L), L.shape[0], L.shape[1], _p(x))
    return x


def symv_lower(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x for symmetric A given by its lower triangle, compensated sums."""
    A = _c(A)
    x = _c(x)
    y = np.empty(A.shape[0])
    _load().oracle_symv_lower(_p(A), A.shape[0], A.shape[1], _p(x), _p(y))
    return y
