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
