"""FP64 CPU oracle for the symmetric sparse kernels (SSYMV, SYPRD, MTTKRP).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports it and it never imports the GPU library; the two share no code.

The oracle evaluates each kernel by its plain definition over the fully
permutation-expanded tensor (SySTeC, arXiv 2406.09266: symmetry and canonical
coordinates, Sec. 2.1; one update per distinct permutation of a stored tuple,
Sec. 3.1; kernel definitions, Sec. 5.2.1, 5.2.3 and 5.2.6). The arithmetic
lives in ``systec_oracle.cpp``; this module builds it with g++ and marshals
numpy arrays to it.

Parity pins (tests/test_oracle_*.py) tie it to the paper's printed 3-D
worked example, dense brute force, the rank-1 closed form, scipy, and
enumeration and invariance properties. The one unpinned quantity is the
magnitude of BF16 rounding error in a full kernel (no closed form); the
rounding of single values is pinned against torch's own conversion.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "systec_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_ORDER = 5


class OracleCounts(ctypes.Structure):
    _fields_ = [
        ("entries", ctypes.c_int64),
        ("effective_nnz", ctypes.c_int64),
        ("noncanonical", ctypes.c_int64),
        ("hist", ctypes.c_int64 * 16),
    ]

    def as_dict(self, order: int) -> dict:
        return {
            "entries": int(self.entries),
            "effective_nnz": int(self.effective_nnz),
            "noncanonical": int(self.noncanonical),
            "hist": [int(self.hist[m]) for m in range(1 << (order - 1))],
        }


def build(force: bool = True) -> str:
    """Compiles the oracle with g++ (-O2, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
# A test that checks the pins catch planted mistakes points this at a mutant
# build of the oracle (see tests/test_oracle_mutants.py).
_LIB_OVERRIDE = os.environ.get("SYSTEC_ORACLE_LIB")


def _load():
    global _lib
    if _lib is None:
        path = _LIB_OVERRIDE or _LIB
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB)
                                  or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_expand.argtypes = [ctypes.c_int, i64, i64, P, P, P, i64, P]
        lib.oracle_mttkrp.argtypes = [ctypes.c_int, i64, i64, P, P, i64, P, ctypes.c_int, P, P, P]
        lib.oracle_ssymv.argtypes = [i64, P, P, P, P, P, P, P]
        lib.oracle_syprd.argtypes = [i64, P, P, P, P, P, P, P]
        lib.oracle_round_bf16.argtypes = [P, P, i64]
        for f in (lib.oracle_expand, lib.oracle_mttkrp, lib.oracle_ssymv, lib.oracle_syprd,
                  lib.oracle_round_bf16):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc == 1:
        raise ValueError(f"oracle {what}: invalid argument or index out of range")
    if rc == 2:
        raise AssertionError(f"oracle {what}: permutation count differs from N!/prod(m!)")
    if rc != 0:
        raise RuntimeError(f"oracle {what}: status {rc}")


def _entry_major(idx, order):
    """Accepts (nnz, order) or a list of `order` index arrays (SoA)."""
    if isinstance(idx, (list, tuple)):
        a = np.stack([np.asarray(v, dtype=np.int32) for v in idx], axis=1)
    else:
        a = np.asarray(idx, dtype=np.int32)
    a = np.ascontiguousarray(a.reshape(-1, order), dtype=np.int32)
    return a


def expand(order, dim, idx, *, coords_cap=0, per_entry=False):
    """Expansion counts; optionally the expanded coordinate list."""
    lib = _load()
    a = _entry_major(idx, order)
    nnz = a.shape[0]
    counts = OracleCounts()
    pc = np.zeros(nnz, dtype=np.int64) if per_entry else None
    coords = np.zeros((coords_cap, order), dtype=np.int32) if coords_cap else None
    rc = lib.oracle_expand(order, dim, nnz, _ptr(a), _ptr(pc), _ptr(coords), coords_cap,
                           ctypes.byref(counts))
    _check(rc, "expand")
    out = counts.as_dict(order)
    if per_entry:
        out["per_entry"] = pc
    if coords_cap:
        out["coords"] = coords[: min(coords_cap, out["effective_nnz"])]
    return out


def mttkrp(order, dim, idx, val, B, *, out_slot=0, row_mask=None):
    """C[i,:] = sum over the expanded tensor (FP64). Returns (C, counts)."""
    lib = _load()
    a = _entry_major(idx, order)
    v = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
    Bm = np.ascontiguousarray(B, dtype=np.float64)
    if Bm.ndim == 1:
        Bm = Bm.reshape(-1, 1)
    R = Bm.shape[1]
    assert Bm.shape[0] == dim and v.shape[0] == a.shape[0]
    C = np.empty((dim, R), dtype=np.float64)
    m = None if row_mask is None else np.ascontiguousarray(row_mask, dtype=np.uint8)
    counts = OracleCounts()
    rc = lib.oracle_mttkrp(order, dim, a.shape[0], _ptr(a), _ptr(v), R, _ptr(Bm), out_slot,
                           _ptr(m), _ptr(C), ctypes.byref(counts))
    _check(rc, "mttkrp")
    return C, counts.as_dict(order)


def _csr(n, rowptr, col, val):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    assert rp.shape[0] == n + 1 and c.shape[0] == v.shape[0] == rp[-1]
    return rp, c, v


def ssymv(n, rowptr, col, val, x, *, row_mask=None):
    """y = A x over the expanded matrix (FP64). Returns (y, counts)."""
    lib = _load()
    rp, c, v = _csr(n, rowptr, col, val)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    m = None if row_mask is None else np.ascontiguousarray(row_mask, dtype=np.uint8)
    counts = OracleCounts()
    rc = lib.oracle_ssymv(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(m), _ptr(y),
                          ctypes.byref(counts))
    _check(rc, "ssymv")
    return y, counts.as_dict(2)


def syprd(n, rowptr, col, val, x):
    """s = x^T A x over the expanded matrix (FP64). Returns (s, abs_s, counts)."""
    lib = _load()
    rp, c, v = _csr(n, rowptr, col, val)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    s = ctypes.c_double()
    sa = ctypes.c_double()
    counts = OracleCounts()
    rc = lib.oracle_syprd(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), ctypes.byref(s),
                          ctypes.byref(sa), ctypes.byref(counts))
    _check(rc, "syprd")
    return s.value, sa.value, counts.as_dict(2)


def round_bf16(x):
    """Rounds FP32 values to bfloat16 (nearest, ties to even); returns FP64."""
    lib = _load()
    a = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(a.shape, dtype=np.float64)
    rc = lib.oracle_round_bf16(_ptr(a), _ptr(out), a.size)
    _check(rc, "round_bf16")
    return out
