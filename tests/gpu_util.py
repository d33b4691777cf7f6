"""Shared helpers of the GPU parity tests (device plumbing and error metrics)."""
from __future__ import annotations

import numpy as np


def rel_l2_per_cell(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """||a_c - b_c||_2 / ||b_c||_2 for every cell c (first axis)."""
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def to_dev(x, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
