"""Helpers for the GPU parity tests."""
import numpy as np


def rel_err(x, ref):
    """Normwise max relative error max|x - ref| / max|ref|."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(x - ref)) / (den if den > 0 else 1.0))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()
