"""Loader for the C oracle (``oracle/c/edm_oracle.c``).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

``build()`` compiles the C file with gcc (-O2, OpenMP, no fast-math) into
``oracle/c/liboracle.so``; ``load()`` builds it on first use if it is
missing and returns a thin numpy-facing wrapper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "edm_oracle.c")
LIB = os.path.join(_HERE, "c", "liboracle.so")

_lib: Optional[ctypes.CDLL] = None


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-fno-fast-math", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    lib = ctypes.CDLL(LIB)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_edm_rows_f64.argtypes = [vp, i64, i32, i64, vp, i64, vp, vp]
    lib.oracle_edm_packed_f64.argtypes = [vp, i64, i32, i64, vp]
    lib.oracle_edm_backward_f64.argtypes = [vp, i64, i32, i64, vp, vp]
    for f in (lib.oracle_edm_rows_f64, lib.oracle_edm_packed_f64,
              lib.oracle_edm_backward_f64):
        f.restype = None
    _lib = lib
    return lib


def _f32(X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be (N, d)")
    return X


def threads() -> int:
    return int(load().oracle_threads())


def edm_rows(X: np.ndarray, rows: Sequence[int]) -> list:
    """Rows of the FP64 triangle (row i has i+1 entries), C loops."""
    X = _f32(X)
    N, d = X.shape
    rows_a = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    lens = rows_a + 1
    off = np.zeros(len(rows_a) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    out = np.empty(int(off[-1]), dtype=np.float64)
    if len(rows_a):
        if rows_a.min() < 0 or rows_a.max() >= N:
            raise ValueError("row out of range")
        load().oracle_edm_rows_f64(X.ctypes.data, N, d, d, rows_a.ctypes.data,
                                   len(rows_a), off.ctypes.data, out.ctypes.data)
    return [out[off[r]: off[r + 1]] for r in range(len(rows_a))]


def edm_packed(X: np.ndarray) -> np.ndarray:
    X = _f32(X)
    N, d = X.shape
    out = np.empty(N * (N + 1) // 2, dtype=np.float64)
    load().oracle_edm_packed_f64(X.ctypes.data, N, d, d, out.ctypes.data)
    return out


def edm_backward(X: np.ndarray, dD_packed: np.ndarray) -> np.ndarray:
    X = _f32(X)
    N, d = X.shape
    dD = np.ascontiguousarray(dD_packed, dtype=np.float32)
    if dD.shape[0] != N * (N + 1) // 2:
        raise ValueError("dD must hold N(N+1)/2 packed cells")
    dX = np.empty((N, d), dtype=np.float64)
    load().oracle_edm_backward_f64(X.ctypes.data, N, d, d, dD.ctypes.data,
                                   dX.ctypes.data)
    return dX
