"""Shared test helpers: seeded inputs on both sides, error norms."""
import numpy as np


def rel_inf(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    s = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / (s if s > 0 else 1.0))


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
