"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import numpy as np


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
