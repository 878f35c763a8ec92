"""Shared helpers of the GPU tests (comparison metrics, device transfer)."""
import numpy as np


def normrel(a, b, mask=None):
    """Per-field norm-relative difference max|a-b| / max|b| over the compared
    points (pointwise relative error is meaningless where a field crosses 0).
    A field whose reference is identically 0 reports max|a-b| instead."""
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a = a[:, mask]
        b = b[:, mask]
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    d = np.abs(a - b).max(axis=1)
    s = np.abs(b).max(axis=1)
    return np.where(s > 0, d / np.where(s > 0, s, 1.0), d)


def to_dev(u):
    import torch
    return torch.as_tensor(np.ascontiguousarray(u), dtype=torch.float64, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def pi_mirror_equal(u, parity):
    return np.array_equal(u, u[:, :, ::-1, ::-1] * parity[:, None, None, None])
