"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, rejects bad arguments before touching the GPU, and its host
canonicalization helper matches a numpy reference. No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2406_09266_amd as systec
from paper_2406_09266_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_symbols():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        names |= set(re.findall(r"SYSTEC_API\s+[\w\s\*]*?\b(systec_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    names = declared_symbols()
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names <= set(_lib.SIGNATURES), "binding lacks a declared entry point"


def test_version_and_no_error():
    assert systec.version().startswith("systec")
    assert _lib.lib().systec_last_error() == b"" or isinstance(_lib.lib().systec_last_error(), bytes)


def _rc(name, *args):
    return getattr(_lib.lib(), name)(*args)


def test_invalid_arguments_are_rejected_on_host():
    P = ctypes.c_void_p
    one = P(16)  # never dereferenced: every call below fails its host checks first
    null = P(0)
    # n < 1
    assert _rc("systec_ssymv", 0, 0, one, one, one, one, 0, one, null) == 1
    # bad dtype
    assert _rc("systec_ssymv", 4, 1, one, one, one, one, 7, one, null) == 1
    # NULL col/val with nnz > 0
    assert _rc("systec_ssymv", 4, 3, one, null, null, one, 0, one, null) == 1
    # NULL output
    assert _rc("systec_syprd", 4, 3, one, one, one, one, 0, null, null) == 1
    # vertex order other than caller (0) or stored (1); NULL prepared handle
    assert _rc("systec_ssymv_t_ex", one, one, 0, one, 7, null) == 1
    assert _rc("systec_syprd_t_ex", one, one, 0, one, -1, null) == 1
    assert _rc("systec_ssymv_t_ex", null, one, 0, one, 1, null) == 1
    assert _rc("systec_syprd_t", null, one, 0, one, null) == 1
    assert _rc("systec_tensor_vertex_order", null, None, null, null) == 1
    # order out of range (symmetric MTTKRP needs 3..5)
    pp, keep = _lib.ptr_array([16, 16, 16, 16, 16, 16])
    assert _rc("systec_mttkrp", 2, 10, 5, pp, one, one, 0, 4, one, null) == 1
    assert _rc("systec_mttkrp", 6, 10, 5, pp, one, one, 0, 4, one, null) == 1
    # R < 1, I*R too large
    assert _rc("systec_mttkrp", 3, 10, 5, pp, one, one, 0, 0, one, null) == 1
    assert _rc("systec_mttkrp", 3, 1 << 20, 5, pp, one, one, 0, 1 << 12, one, null) == 1
    # nnz >= 2^31
    assert _rc("systec_mttkrp", 3, 10, 1 << 31, pp, one, one, 0, 4, one, null) == 1
    msg = _lib.lib().systec_last_error().decode()
    assert "nnz" in msg
    # NULL index pointer
    pn, keep2 = _lib.ptr_array([16, 0, 16])
    assert _rc("systec_mttkrp", 3, 10, 5, pn, one, one, 0, 4, one, null) == 1
    # quantize: negative size
    assert _rc("systec_quantize_bf16", one, one, -1, null) == 1
    with pytest.raises(systec.SystecError) as e:
        _lib.call("systec_ssymv", 0, 0, one, one, one, one, 0, one, null)
    assert e.value.status_name == "SYSTEC_EINVAL"
    del keep, keep2


def test_canonicalize_coo_matches_numpy():
    rng = np.random.Generator(np.random.PCG64(7))
    order, dim, n = 4, 9, 3000
    raw = rng.integers(0, dim, (n, order)).astype(np.int32)
    val = rng.standard_normal(n)
    idx = [np.ascontiguousarray(raw[:, t]) for t in range(order)]
    v = val.copy()
    m = systec.canonicalize_coo(idx, v)
    # numpy reference: sort tuples, group equal tuples, sum
    srt = np.sort(raw, axis=1)
    keys = np.zeros(n, dtype=np.int64)
    for t in range(order):
        keys = keys * dim + srt[:, t]
    uk, inv = np.unique(keys, return_inverse=True)
    sums = np.zeros(uk.size)
    np.add.at(sums, inv, val)
    assert m == uk.size
    got = np.stack([a[:m] for a in idx], axis=1).astype(np.int64)
    gk = np.zeros(m, dtype=np.int64)
    for t in range(order):
        gk = gk * dim + got[:, t]
    assert np.array_equal(gk, uk)
    np.testing.assert_allclose(v[:m], sums, rtol=1e-13, atol=1e-13)


def test_canonicalize_keeps_canonical_input():
    t = synth.sym_coo(3, 50, 500, 0.1, seed=5)
    idx = [np.ascontiguousarray(a) for a in t["idx"]]
    v = t["val"].copy()
    assert systec.canonicalize_coo(idx, v) == 500
    assert all(np.array_equal(a, b) for a, b in zip(idx, t["idx"]))
    assert np.array_equal(v, t["val"])
