"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def to_dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def to_host(T):
    return T.detach().cpu().numpy()


def frob_err(a, b):
    """||a - b||_F / ||b||_F over the whole block."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_err(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: element by element, so one wrong
    coefficient counts in full however large the block."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def rel_err(a, b):
    """The larger of the element-wise (max_err) and whole-block (frob_err)
    relative errors; a parity bar holds for both."""
    return max(frob_err(a, b), max_err(a, b))
