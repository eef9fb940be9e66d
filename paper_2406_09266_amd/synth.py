"""Seeded synthetic inputs for the symmetric sparse kernels.

This module draws random inputs only. It holds none of the method's
arithmetic (no permutation expansion, no multiplicities, no coefficients), so
that the FP64 oracle and the GPU library can both be fed from it without
sharing any computation.

Every generator takes an explicit seed and uses numpy's PCG64, so a seed
reproduces byte-identical arrays. All outputs are canonical: a stored tuple
ascends (c1 <= ... <= cN, the upper triangle for matrices), the list is sorted
lexicographically and holds no duplicate tuple. Indices are 0-based int32.

Shapes follow the paper's workloads (SySTeC, arXiv 2406.09266, Sec. 5.2):
symmetric sparse matrices for SSYMV and SYPRD, and uniformly random
(Erdos-Renyi) symmetric sparse tensors with dense random factors for MTTKRP.
The paper's matrix suite and tensor files are not available; these generators
stand in for them with the same structure.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Matrices (CSR of the upper triangle, diagonal included)
# --------------------------------------------------------------------------

def _csr_from_sorted_keys(n, rows, cols):
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.bincount(rows.astype(np.int64), minlength=n)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return rowptr, cols.astype(np.int32)


def ssymv_uniform(n, offdiag_per_row=9, seed=1, with_diagonal=True):
    """Upper-triangle CSR: row i stores (i, i) and min(k, n-1-i) distinct
    columns drawn uniformly without replacement from (i, n).
    Values N(0,1) FP64, x U(-1,1) FP64."""
    rng = _rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = min(offdiag_per_row, n - 1 - i)
        c = (rng.choice(n - 1 - i, size=k, replace=False) + i + 1) if k > 0 else np.empty(0, np.int64)
        if with_diagonal:
            c = np.concatenate([[i], c])
        c = np.sort(c)
        rows.append(np.full(c.size, i, dtype=np.int64))
        cols.append(c.astype(np.int64))
    rows = np.concatenate(rows) if rows else np.empty(0, np.int64)
    cols = np.concatenate(cols) if cols else np.empty(0, np.int64)
    rowptr, col = _csr_from_sorted_keys(n, rows, cols)
    val = rng.standard_normal(col.size)
    x = rng.uniform(-1.0, 1.0, n)
    return {"n": n, "rowptr": rowptr, "col": col, "val": val, "x": x}


def ssymv_rmat(scale=22, a=0.57, b=0.19, c=0.19, avg_degree=16, batch=1 << 22, seed=2,
               relabel=False):
    """Symmetric R-MAT adjacency, upper-triangle CSR.

    Each edge takes `scale` quadrant choices with probabilities (a, b, c, d).
    An edge maps to (min, max); self-loops are kept; duplicates merge. Edges are
    drawn in batches of `batch` until the full matrix holds at least
    avg_degree * n entries (2 U - D, U stored, D on the diagonal); the whole
    last batch is kept. Values U(0,1) per unique entry in sorted order,
    x U(-1,1). With relabel=True a seeded random vertex permutation is applied
    first (moves the hubs away from low indices)."""
    n = 1 << scale
    rng = _rng(seed)
    perm = rng.permutation(n).astype(np.int64) if relabel else None
    ab, abc = a + b, a + b + c
    keys = np.empty(0, dtype=np.int64)
    while True:
        src = np.zeros(batch, dtype=np.int64)
        dst = np.zeros(batch, dtype=np.int64)
        for _ in range(scale):
            u = rng.random(batch, dtype=np.float32)
            rbit = (u >= ab).astype(np.int64)                     # quadrants c, d
            cbit = (((u >= a) & (u < ab)) | (u >= abc)).astype(np.int64)  # quadrants b, d
            src = (src << 1) | rbit
            dst = (dst << 1) | cbit
        if perm is not None:
            src, dst = perm[src], perm[dst]
        lo = np.minimum(src, dst)
        hi = np.maximum(src, dst)
        new = np.unique((lo << scale) | hi)
        merged = np.sort(np.concatenate([keys, new]), kind="stable")
        keep = np.ones(merged.size, dtype=bool)
        keep[1:] = merged[1:] != merged[:-1]
        keys = merged[keep]
        rows = keys >> scale
        cols = keys & (n - 1)
        d = int(np.count_nonzero(rows == cols))
        if 2 * keys.size - d >= avg_degree * n:
            break
    rowptr, col = _csr_from_sorted_keys(n, rows, cols)
    val = rng.uniform(0.0, 1.0, col.size)
    x = rng.uniform(-1.0, 1.0, n)
    return {"n": n, "rowptr": rowptr, "col": col, "val": val, "x": x,
            "diag": d}


def ssymv_random_degree(n, avg_degree, seed):
    """Upper-triangle CSR with uniformly random columns, about avg_degree
    entries per row of the full matrix; values U(0,1), x U(-1,1)."""
    rng = _rng(seed)
    m = max(1, int(round(avg_degree * n / 2)))
    i = rng.integers(0, n, m, dtype=np.int64)
    j = rng.integers(0, n, m, dtype=np.int64)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    keys = np.unique(lo * n + hi)
    rows, cols = keys // n, keys % n
    rowptr, col = _csr_from_sorted_keys(n, rows, cols)
    val = rng.uniform(0.0, 1.0, col.size)
    x = rng.uniform(-1.0, 1.0, n)
    return {"n": n, "rowptr": rowptr, "col": col, "val": val, "x": x}


# --------------------------------------------------------------------------
# Symmetric sparse tensors (canonical COO, structure of arrays)
# --------------------------------------------------------------------------

def compositions(order):
    """Ordered run-length compositions of `order` (e.g. 3 -> (1,1,1), (1,2),
    (2,1), (3)); a composition describes which adjacent indices of a sorted
    tuple are equal."""
    out = []
    for cuts in itertools.product([0, 1], repeat=order - 1):
        runs, run = [], 1
        for cut in cuts:
            if cut:
                run += 1
            else:
                runs.append(run)
                run = 1
        runs.append(run)
        out.append(tuple(runs))
    return sorted(set(out), key=lambda r: (-len(r), r))


def _keys(tuples, dim):
    """Mixed-radix int64 keys of sorted tuples (lexicographic order)."""
    k = np.zeros(tuples.shape[0], dtype=np.int64)
    for t in range(tuples.shape[1]):
        k = k * dim + tuples[:, t]
    return k


def _draw_distinct_sorted(rng, count, k, dim):
    """`count` sorted tuples of k pairwise different values in [0, dim)."""
    out = np.empty((0, k), dtype=np.int64)
    while out.shape[0] < count:
        need = count - out.shape[0]
        t = rng.integers(0, dim, (need + need // 8 + 16, k), dtype=np.int64)
        t.sort(axis=1)
        ok = np.all(t[:, 1:] != t[:, :-1], axis=1) if k > 1 else np.ones(t.shape[0], bool)
        out = np.concatenate([out, t[ok][:need]])
    return out


def _unique_class(rng, count, comp, dim, order):
    """`count` unique sorted tuples with the run-length composition `comp`."""
    k = len(comp)
    reps = np.array(comp)
    got = np.empty((0, order), dtype=np.int64)
    while got.shape[0] < count:
        need = count - got.shape[0]
        base = _draw_distinct_sorted(rng, need, k, dim)
        tup = np.repeat(base, reps, axis=1)
        got = np.concatenate([got, tup])
        _, first = np.unique(_keys(got, dim), return_index=True)
        got = got[np.sort(first)]
    return got[:count]


def sym_coo(order, dim, nnz, repeat_frac, seed, R=None, class_cap=0.5):
    """Random symmetric sparse tensor of the given order in canonical COO.

    A fraction 1 - repeat_frac of the entries has pairwise different indices
    (order iid uniform draws, redrawn on a collision, then sorted). The rest
    has repeated indices: its composition is spread evenly over the repeat
    compositions; a class holds at most class_cap of its possible tuples and
    its overflow moves to the other repeat classes. Tuples are unique and the
    list is sorted lexicographically. Values N(0,1) FP64; if R is given, a
    dense factor B (dim x R) U(-1,1) FP64 is drawn too.

    Returns idx as int32 (order, nnz), val, optional B, and the number of
    entries drawn per composition."""
    rng = _rng(seed)
    comps = [c for c in compositions(order) if len(c) < order]
    n_rep = int(round(nnz * repeat_frac)) if comps else 0
    n_dis = nnz - n_rep
    # split the repeated entries evenly, honoring each class's capacity
    cap = {c: int(class_cap * math.comb(dim, len(c))) for c in comps}
    target = {c: 0 for c in comps}
    left, open_ = n_rep, list(comps)
    while left > 0 and open_:
        share = max(1, left // len(open_))
        for c in list(open_):
            give = min(share, cap[c] - target[c], left)
            target[c] += give
            left -= give
            if target[c] >= cap[c]:
                open_.remove(c)
            if left == 0:
                break
    if left > 0:
        raise ValueError("not enough tuples with repeated indices for the requested fraction")
    if n_dis > math.comb(dim, order):
        raise ValueError("more entries with pairwise different indices requested than exist")
    parts, drawn = [], {}
    # pairwise-different part, unique
    got = np.empty((0, order), dtype=np.int64)
    while got.shape[0] < n_dis:
        got = np.concatenate([got, _draw_distinct_sorted(rng, n_dis - got.shape[0], order, dim)])
        got = got[np.unique(_keys(got, dim), return_index=True)[1]]
    parts.append(got[:n_dis])
    drawn[tuple([1] * order)] = int(n_dis)
    for c in comps:
        if target[c]:
            parts.append(_unique_class(rng, target[c], c, dim, order))
        drawn[c] = int(target[c])
    tup = np.concatenate(parts) if parts else np.empty((0, order), np.int64)
    if float(dim) ** order < 2.0 ** 62:
        tup = tup[np.argsort(_keys(tup, dim), kind="stable")]
    else:
        tup = tup[np.lexsort(tup.T[::-1])]
    idx = np.ascontiguousarray(tup.T.astype(np.int32))
    val = rng.standard_normal(idx.shape[1])
    out = {"order": order, "dim": dim, "idx": idx, "val": val, "drawn": drawn}
    if R is not None:
        out["B"] = rng.uniform(-1.0, 1.0, (dim, R))
    return out


def partial_coo(parts, dim, nnz, repeat_frac, seed, R=None):
    """Random tensor symmetric inside consecutive parts of its slots (part
    sizes `parts`), in canonical COO: indices ascending inside every part,
    tuples unique, the list sorted lexicographically. Uniform iid indices;
    in a fraction repeat_frac of the tuples one random adjacent pair of
    slots inside a part of size >= 2 is made equal (so repeated indices
    occur at every position). Values N(0,1) FP64; with R, one factor
    U(-1,1) (dim x R) per part. At most nnz tuples (duplicates dropped)."""
    rng = _rng(seed)
    order = int(sum(parts))
    t = rng.integers(0, dim, (nnz, order))
    starts = np.cumsum([0] + list(parts[:-1]))
    multi = [(int(s0), int(q)) for s0, q in zip(starts, parts) if q >= 2]
    rep = np.flatnonzero(rng.random(nnz) < repeat_frac) if multi else np.empty(0, np.int64)
    for e in rep:
        start, size = multi[int(rng.integers(0, len(multi)))]
        k = start + int(rng.integers(0, size - 1))
        t[e, k + 1] = t[e, k]
    s0 = 0
    for q in parts:
        t[:, s0:s0 + q] = np.sort(t[:, s0:s0 + q], axis=1)
        s0 += q
    t = np.unique(t, axis=0)  # sorted lexicographically, unique
    idx = np.ascontiguousarray(t.T.astype(np.int32))
    out = {"parts": list(parts), "order": order, "dim": dim, "idx": idx,
           "val": rng.standard_normal(idx.shape[1])}
    if R is not None:
        out["F"] = [rng.uniform(-1.0, 1.0, (dim, R)) for _ in parts]
    return out


def dense_uniform(shape, seed, low=-1.0, high=1.0):
    return _rng(seed).uniform(low, high, shape)


def integer_valued(shape, seed, low=-3, high=3):
    """Small integers as FP64: products and sums of them are exact in FP64
    and, for short sums, in FP32."""
    return _rng(seed).integers(low, high + 1, shape).astype(np.float64)


# --------------------------------------------------------------------------
# The workloads the paper's evaluation is shaped like
# --------------------------------------------------------------------------

def workload(name):
    """Named configurations:

    ssymv_small  n=2,000, ~10 stored entries per row (diagonal included),
                 uniform columns, N(0,1) values                     (seed 1)
    ssymv_rmat   R-MAT scale 22 (n=4,194,304), a,b,c=.57,.19,.19,
                 average degree 16, U(0,1) values                  (seed 2)
    mttkrp3      order 3, I=100,000, 20M canonical entries, 1% with repeated
                 indices, N(0,1) values, B 100,000 x 32            (seed 3)
    mttkrp5      order 5, I=5,000, 5M canonical entries, 5% with repeated
                 indices, N(0,1) values, B 5,000 x 16               (seed 4)
    """
    if name == "ssymv_small":
        return ssymv_uniform(2000, 9, seed=1)
    if name == "ssymv_rmat":
        return ssymv_rmat(scale=22, seed=2)
    if name == "mttkrp3":
        return sym_coo(3, 100_000, 20_000_000, 0.01, seed=3, R=32)
    if name == "mttkrp5":
        return sym_coo(5, 5_000, 5_000_000, 0.05, seed=4, R=16)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Device-side generators (torch on the GPU) for the large serving pool
# --------------------------------------------------------------------------

def _tgen(seed, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def gpu_ssymv_random(n, avg_degree, seed, device="cuda"):
    """Upper-triangle CSR on the device: about avg_degree * n / 2 uniformly
    random edges, mapped to (min, max), duplicates merged; values U(0,1)."""
    import torch
    g = _tgen(seed, device)
    m = max(1, int(round(avg_degree * n / 2)))
    i = torch.randint(0, n, (m,), generator=g, device=device, dtype=torch.int64)
    j = torch.randint(0, n, (m,), generator=g, device=device, dtype=torch.int64)
    keys = torch.unique(torch.minimum(i, j) * n + torch.maximum(i, j))
    rows, cols = keys // n, keys % n
    counts = torch.bincount(rows, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    val = torch.rand(cols.numel(), generator=g, device=device, dtype=torch.float32)
    return {"n": n, "rowptr": rowptr.to(torch.int32), "col": cols.to(torch.int32), "val": val}


def gpu_sym_coo(order, dim, nnz, repeat_frac, seed, device="cuda"):
    """Canonical COO of a random symmetric tensor on the device: iid uniform
    index tuples (a fraction repeat_frac made to repeat one index), sorted
    within each tuple, sorted lexicographically, duplicates removed (so the
    result can hold slightly fewer than nnz entries). Values N(0,1)."""
    import torch
    g = _tgen(seed, device)
    m = int(nnz * 1.05) + 16
    t = torch.randint(0, dim, (m, order), generator=g, device=device, dtype=torch.int64)
    rep = torch.rand(m, generator=g, device=device) < repeat_frac
    k = torch.randint(0, order - 1, (m,), generator=g, device=device)
    rows = torch.nonzero(rep).squeeze(1)
    t[rows, k[rows] + 1] = t[rows, k[rows]]
    t, _ = torch.sort(t, dim=1)
    for c in range(order - 1, -1, -1):  # lexicographic: stable sorts, last key first
        _, p = torch.sort(t[:, c], stable=True)
        t = t[p]
    keep = torch.ones(t.shape[0], dtype=torch.bool, device=device)
    keep[1:] = torch.any(t[1:] != t[:-1], dim=1)
    t = t[keep][:nnz]
    val = torch.randn(t.shape[0], generator=g, device=device, dtype=torch.float32)
    idx = [t[:, c].to(torch.int32).contiguous() for c in range(order)]
    return {"order": order, "dim": dim, "idx": idx, "val": val}
