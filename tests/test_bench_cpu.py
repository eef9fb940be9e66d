"""CPU checks of bench.py's host-side helpers (no GPU): the relabeled matrix
it builds for the comparison kernels is P A P^T of the stored matrix."""
import importlib.util
import os

import numpy as np

from paper_2406_09266_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _dense_sym(n, rowptr, col, val):
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            A[i, col[k]] = A[col[k], i] = val[k]
    return A


def test_degree_ordered_csr_is_the_permuted_matrix():
    import torch
    bench = _bench()
    m = synth.ssymv_rmat(scale=7, batch=1 << 9, seed=61)
    n = m["n"]
    rows = np.repeat(np.arange(n), np.diff(m["rowptr"]))
    col = m["col"].astype(np.int64)
    deg = np.bincount(rows, minlength=n) + np.bincount(col[col != rows], minlength=n)
    perm = np.argsort(-deg, kind="stable")
    rp2, col2, val2 = bench.degree_ordered_csr(
        torch, torch.from_numpy(m["rowptr"]), torch.from_numpy(m["col"]),
        torch.from_numpy(m["val"].astype(np.float32)), torch.from_numpy(perm.astype(np.int32)))
    rp2, col2, val2 = rp2.numpy(), col2.numpy(), val2.numpy()
    # still an upper-triangle CSR with sorted columns
    r2 = np.repeat(np.arange(n), np.diff(rp2))
    assert np.all(col2 >= r2)
    assert all(np.all(np.diff(col2[rp2[i]:rp2[i + 1]]) > 0) for i in range(n))
    A = _dense_sym(n, m["rowptr"], m["col"], m["val"].astype(np.float32))
    B = _dense_sym(n, rp2, col2, val2)
    assert np.array_equal(B, A[np.ix_(perm, perm)])
