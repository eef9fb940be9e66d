"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import numpy as np

from paper_2406_09266_amd import synth


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(got, want):
    """Normwise relative error ||got - want|| / ||want|| (exact zero required
    when want is zero)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want)
    num = np.linalg.norm(got - want)
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def f32(a):
    """The FP32 values the GPU sees, back in FP64 (exact)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def csr_to_dev(m):
    import torch
    return (dev(m["rowptr"]), dev(m["col"]), dev(m["val"].astype(np.float32)),
            dev(m["x"].astype(np.float32)))


def assert_elementwise(got, want, scale, tol, what=""):
    """Every element within tol of the oracle, relative to that element's own
    scale: |got_i - want_i| <= tol * scale_i, where scale_i is the oracle's
    result on the absolute values of the same inputs (the sum of |terms| that
    make up element i). An element with no terms must be exactly zero."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    assert got.shape == want.shape == scale.shape, (got.shape, want.shape, scale.shape)
    diff = np.abs(got - want)
    bad = ~(diff <= tol * scale)
    if bad.any():
        i = np.flatnonzero(bad.reshape(-1))[0]
        raise AssertionError(
            f"{what}: {int(bad.sum())} of {bad.size} elements off; first flat index {i}: "
            f"got {got.reshape(-1)[i]!r} want {want.reshape(-1)[i]!r} "
            f"scale {scale.reshape(-1)[i]!r} (tol {tol})")


def wide_step_matrix():
    """A matrix whose panels mix narrow and wide steps: the first panel is a
    dense band (64 consecutive entries span a few hundred columns), the rest
    hold a few rows with entries spread over the whole column range, so a
    step of 64 sorted entries (padding included) spans more than 2^19
    columns and the kernels take its columns from the unpacked stream."""
    n = 2_000_000
    rng = np.random.Generator(np.random.PCG64(61))
    rows, cols = [], []
    for i in range(4000):  # band rows: 12 entries each within 4,000 columns
        c = np.unique(i + rng.integers(0, 4000, 12))
        rows.append(np.full(c.size, i)); cols.append(c)
    for i in range(5000, n, 6007):  # sparse rows: the diagonal and 3 far columns
        c = np.unique(np.r_[i, rng.integers(i, n, 3)])
        rows.append(np.full(c.size, i)); cols.append(c)
    r = np.concatenate(rows).astype(np.int64); c = np.concatenate(cols).astype(np.int64)
    order = np.lexsort((c, r)); r, c = r[order], c[order]
    rowptr = np.zeros(n + 1, np.int64); np.add.at(rowptr, r + 1, 1); rowptr = np.cumsum(rowptr)
    return {"n": n, "rowptr": rowptr.astype(np.int32), "col": c.astype(np.int32),
            "val": synth.dense_uniform(c.size, seed=62, low=0.0, high=1.0),
            "x": synth.dense_uniform(n, seed=63)}
