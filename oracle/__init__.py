"""FP64 CPU oracle for the symmetric sparse kernels (SSYMV, SYPRD, MTTKRP,
and next to them the Bellman-Ford update, TTM, MTTKRP of a partially
symmetric tensor and the symmetric CP step).

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
imports it and it never imports the GPU library; the two share no code.

The oracle evaluates each kernel by its plain definition over the fully
permutation-expanded tensor (SySTeC, arXiv 2406.09266: symmetry and canonical
coordinates, Sec. 2.1; one update per distinct permutation of a stored tuple,
Sec. 3.1; kernel definitions, Sec. 5.2.1, 5.2.2, 5.2.3, 5.2.5 and 5.2.6;
partial symmetry, Sec. 2.1). The arithmetic over the expanded tensor lives in
``systec_oracle.cpp``; this module builds it with g++ and marshals numpy
arrays to it. The CP step (``cp_step``) composes the oracle's MTTKRP with
dense FP64 linear algebra in numpy.

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
            ["g++", "-O2", "-std=c++17", "-fPIC", "-fopenmp", "-shared", "-o", tmp, _SRC])
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
        lib.oracle_mttkrp_mt.argtypes = lib.oracle_mttkrp.argtypes + [ctypes.c_int]
        lib.oracle_ssymv_mt.argtypes = lib.oracle_ssymv.argtypes + [ctypes.c_int]
        lib.oracle_threads.argtypes = []
        lib.oracle_bellman_ford.argtypes = [i64, P, P, P, P, P, P]
        lib.oracle_ttm3.argtypes = [i64, i64, P, P, i64, P, P, P]
        lib.oracle_mttkrp_partial.argtypes = [ctypes.c_int, ctypes.c_int, P, i64, i64, P, P, i64,
                                              P, P, P]
        for f in (lib.oracle_expand, lib.oracle_mttkrp, lib.oracle_ssymv, lib.oracle_syprd,
                  lib.oracle_round_bf16, lib.oracle_mttkrp_mt, lib.oracle_ssymv_mt,
                  lib.oracle_threads, lib.oracle_bellman_ford, lib.oracle_ttm3,
                  lib.oracle_mttkrp_partial):
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


def threads():
    """The number of host threads the all-core variants use by default."""
    return int(_load().oracle_threads())


def mttkrp(order, dim, idx, val, B, *, out_slot=0, row_mask=None, threads=1):
    """C[i,:] = sum over the expanded tensor (FP64). Returns (C, counts).
    threads > 1 (or 0: every core) splits the stored entries statically over
    host threads with private FP64 outputs summed in thread order."""
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
    rc = lib.oracle_mttkrp_mt(order, dim, a.shape[0], _ptr(a), _ptr(v), R, _ptr(Bm), out_slot,
                              _ptr(m), _ptr(C), ctypes.byref(counts), int(threads))
    _check(rc, "mttkrp")
    return C, counts.as_dict(order)


def _csr(n, rowptr, col, val):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    assert rp.shape[0] == n + 1 and c.shape[0] == v.shape[0] == rp[-1]
    return rp, c, v


def ssymv(n, rowptr, col, val, x, *, row_mask=None, threads=1):
    """y = A x over the expanded matrix (FP64). Returns (y, counts).
    threads as for mttkrp."""
    lib = _load()
    rp, c, v = _csr(n, rowptr, col, val)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    m = None if row_mask is None else np.ascontiguousarray(row_mask, dtype=np.uint8)
    counts = OracleCounts()
    rc = lib.oracle_ssymv_mt(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), _ptr(m), _ptr(y),
                             ctypes.byref(counts), int(threads))
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


def bellman_ford(n, rowptr, col, val, d):
    """y[i] = min_j (A[i,j] + d[j]) over the stored coordinates of the
    expanded matrix (FP64; +inf where row i has none). Returns (y, counts)."""
    lib = _load()
    rp, c, v = _csr(n, rowptr, col, val)
    dd = np.ascontiguousarray(d, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    counts = OracleCounts()
    rc = lib.oracle_bellman_ford(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(dd), _ptr(y),
                                 ctypes.byref(counts))
    _check(rc, "bellman_ford")
    return y, counts.as_dict(2)


def ttm3(dim, idx, val, B):
    """C[j, l, r] = sum_k A[k, j, l] B[k, r] over the expanded symmetric
    3-index tensor A (FP64). Returns (C of shape (dim, dim, R), counts)."""
    lib = _load()
    a = _entry_major(idx, 3)
    v = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
    Bm = np.ascontiguousarray(B, dtype=np.float64)
    R = Bm.shape[1]
    assert Bm.shape[0] == dim and v.shape[0] == a.shape[0]
    C = np.empty((dim, dim, R), dtype=np.float64)
    counts = OracleCounts()
    rc = lib.oracle_ttm3(dim, a.shape[0], _ptr(a), _ptr(v), R, _ptr(Bm), _ptr(C),
                         ctypes.byref(counts))
    _check(rc, "ttm3")
    return C, counts.as_dict(3)


def mttkrp_partial(parts, dim, idx, val, F):
    """MTTKRP (output mode 1) of a tensor symmetric only inside each part of
    its slots: parts lists the sizes of consecutive slot groups (e.g. [2, 2]
    for slots {1,2},{3,4}); F lists one dim x R factor per part. Returns
    (C, counts)."""
    lib = _load()
    parts = [int(q) for q in parts]
    order = sum(parts)
    a = _entry_major(idx, order)
    v = np.ascontiguousarray(val, dtype=np.float64).reshape(-1)
    Fm = np.ascontiguousarray(np.stack([np.asarray(f, dtype=np.float64) for f in F]))
    assert Fm.shape[0] == len(parts) and Fm.shape[1] == dim
    R = Fm.shape[2]
    ps = np.array(parts, dtype=np.int32)
    C = np.empty((dim, R), dtype=np.float64)
    counts = OracleCounts()
    rc = lib.oracle_mttkrp_partial(order, len(parts), _ptr(ps), dim, a.shape[0], _ptr(a), _ptr(v),
                                   R, _ptr(Fm), _ptr(C), ctypes.byref(counts))
    _check(rc, "mttkrp_partial")
    return C, counts.as_dict(order)


def cp_step(order, dim, idx, val, B, threads=1):
    """One step of symmetric CP-ALS around MTTKRP (Sec. 5.2.6: the symmetric
    CPD uses one factor matrix B for every mode, so the update is the same in
    every mode), in FP64:

        C      = MTTKRP(T, B)                      (the oracle's, expanded T)
        G      = B^T B
        H      = G^(N-1), elementwise (the Gram matrix of the Khatri-Rao
                 product of N-1 copies of B)
        B_new  = C H^-1                            (the least-squares update)
        fit terms of the model [[B]] = sum_r b_r^(x N):
          norm_T2 = ||T||^2        = sum over stored entries of
                                     (distinct permutations) * v^2
          inner   = <T, [[B]]>     = sum_{i,r} C[i,r] B[i,r]
          norm_M2 = ||[[B]]||^2    = sum_{r,s} G[r,s]^N
          resid2  = ||T - [[B]]||^2 = norm_T2 - 2 inner + norm_M2
    Returns a dict of these."""
    Bm = np.asarray(B, dtype=np.float64)
    C, counts = mttkrp(order, dim, idx, val, Bm, threads=threads)
    G = Bm.T @ Bm
    H = G ** (order - 1)
    B_new = np.linalg.solve(H, C.T).T  # H is symmetric: B_new H = C
    per = expand(order, dim, idx, per_entry=True)["per_entry"]
    v = np.asarray(val, dtype=np.float64).reshape(-1)
    norm_T2 = float(np.sum(per * v * v))
    inner = float(np.sum(C * Bm))
    norm_M2 = float(np.sum(G ** order))
    return {"C": C, "G": G, "H": H, "B_new": B_new, "norm_T2": norm_T2, "inner": inner,
            "norm_M2": norm_M2, "resid2": norm_T2 - 2.0 * inner + norm_M2, "counts": counts}

