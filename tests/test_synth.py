"""Seeded generators: reproducible, canonical, sorted, duplicate-free."""
import numpy as np
import pytest

from paper_2406_09266_amd import synth


def _check_csr_upper(m):
    n, rp, col = m["n"], m["rowptr"], m["col"]
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(col >= rows) and np.all(col < n)
    key = rows.astype(np.int64) * n + col
    assert np.all(np.diff(key) > 0)  # sorted, unique


def test_ssymv_uniform_shape_and_seed():
    a = synth.ssymv_uniform(300, 9, seed=1)
    b = synth.ssymv_uniform(300, 9, seed=1)
    for k in ("rowptr", "col", "val", "x"):
        assert np.array_equal(a[k], b[k])
    _check_csr_upper(a)
    deg = np.diff(a["rowptr"])
    assert np.all(deg == 1 + np.minimum(9, 300 - 1 - np.arange(300)))


def test_ssymv_rmat_small():
    m = synth.ssymv_rmat(scale=12, batch=1 << 14, seed=2)
    _check_csr_upper(m)
    n = m["n"]
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    d = int(np.count_nonzero(rows == m["col"]))
    assert 2 * m["col"].size - d >= 16 * n
    m2 = synth.ssymv_rmat(scale=12, batch=1 << 14, seed=2)
    assert np.array_equal(m["col"], m2["col"]) and np.array_equal(m["val"], m2["val"])


@pytest.mark.parametrize("order,dim,nnz,frac", [(3, 1000, 20000, 0.01), (4, 300, 20000, 0.05),
                                                (5, 200, 20000, 0.05)])
def test_sym_coo_canonical(order, dim, nnz, frac):
    t = synth.sym_coo(order, dim, nnz, frac, seed=3, R=4)
    idx = t["idx"]
    assert idx.dtype == np.int32 and idx.shape == (order, nnz)
    assert np.all(np.diff(idx, axis=0) >= 0)
    assert idx.min() >= 0 and idx.max() < dim
    key = np.zeros(nnz, dtype=np.int64)
    for r in range(order):
        key = key * dim + idx[r]
    assert np.all(np.diff(key) > 0)
    rep = np.any(np.diff(idx, axis=0) == 0, axis=0).sum()
    assert rep == round(nnz * frac)
    assert sum(t["drawn"].values()) == nnz
    t2 = synth.sym_coo(order, dim, nnz, frac, seed=3, R=4)
    assert np.array_equal(t2["idx"], idx) and np.array_equal(t2["B"], t["B"])


def test_compositions():
    assert synth.compositions(3) == [(1, 1, 1), (1, 2), (2, 1), (3,)]
    assert len(synth.compositions(5)) == 16
