"""Helpers for the GPU parity tests (no method arithmetic here)."""
import numpy as np


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def to_dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rounded(a, dtype):
    """The values a GPU run of this dtype actually receives, as float64."""
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype).double().numpy()
