"""The method's symmetric loops on one host core (FP64), for the benchmark's
CPU analog of the paper's symmetric-against-naive comparison: SSYMV over the
stored upper triangle (SySTeC, arXiv 2406.09266, Sec. 3.1) and MTTKRP over
canonical tuples with the count of each value's distinct permutations
(Sec. 4.2.5, 4.2.7, 5.2.6).

TEST INFRASTRUCTURE (benchmark baseline) ONLY. Only the test suite and the
benchmark's CPU-baseline leg may import this module. These loops are not the
oracle and decide no parity question; tests/test_host_loops.py pins them to
the oracle's expanded definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "host_loops.cpp")
_LIB = os.path.join(_HERE, "libhostloops.so")
_lib = None


def build(force: bool = True) -> str:
    """Compiles the loops with g++ (-O2, no fast-math, one thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.host_ssymv_canonical.argtypes = [i64, P, P, P, P, P]
        lib.host_mttkrp_canonical.argtypes = [ctypes.c_int, i64, i64, P, P, P, i64, P]
        lib.host_ssymv_canonical.restype = ctypes.c_int
        lib.host_mttkrp_canonical.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def ssymv(n, rowptr, col, val, x):
    """y = A x from the canonical upper-triangle CSR, FP64."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    if _load().host_ssymv_canonical(n, _p(rp), _p(cl), _p(v), _p(xx), _p(y)) != 0:
        raise ValueError("host ssymv: invalid argument or index")
    return y


def mttkrp(order, dim, idx, val, B):
    """C = MTTKRP of the symmetric tensor from its canonical tuples; idx is
    (nnz, order) entry-major, ascending within a tuple. FP64."""
    ix = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, order)
    v = np.ascontiguousarray(val, dtype=np.float64)
    Bm = np.ascontiguousarray(B, dtype=np.float64)
    R = Bm.shape[1]
    C = np.empty((dim, R), dtype=np.float64)
    rc = _load().host_mttkrp_canonical(order, dim, ix.shape[0], _p(ix), _p(v), _p(Bm), R, _p(C))
    if rc != 0:
        raise ValueError("host mttkrp: invalid argument or index")
    return C
