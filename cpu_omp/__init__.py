"""Multi-core CPU baseline (OpenMP CSR, Sec. IV-A): measurement infrastructure,
not an oracle and not part of the GPU library (it shares no code with either).

Only bench.py and the tests load it. Rows are split into contiguous blocks of
equal nonzero counts, one per thread; the thread count is OpenMP's default
(OMP_NUM_THREADS when set, else every core)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_omp.c")
_LIB = os.path.join(_HERE, "libcsromp.so")
_lib = None

# generic x86-64 code (the library travels to other hosts)
GCC_FLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        L.omp_spmv.restype = None
        L.omp_spmv.argtypes = [i32, P, P, P, P, P]
        L.omp_spmv_time.restype = ctypes.c_double
        L.omp_spmv_time.argtypes = [i32, P, P, P, P, P, i32, P]
        _lib = L
    return _lib


def _arrays(rp, col, val, x):
    return (np.ascontiguousarray(rp, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64), np.ascontiguousarray(x, dtype=np.float64))


def spmv(rp, col, val, x) -> np.ndarray:
    rp, col, val, x = _arrays(rp, col, val, x)
    n = rp.size - 1
    y = np.empty(n, dtype=np.float64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    lib().omp_spmv(n, p(rp), p(col), p(val), p(x), p(y))
    return y


def time_spmv(rp, col, val, x, calls: int):
    """(seconds for `calls` products, threads used)."""
    rp, col, val, x = _arrays(rp, col, val, x)
    n = rp.size - 1
    y = np.empty(n, dtype=np.float64)
    th = ctypes.c_int32(0)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    sec = lib().omp_spmv_time(n, p(rp), p(col), p(val), p(x), p(y), calls, ctypes.byref(th))
    return sec, th.value
