"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def to_dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def to_host(T):
    return T.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
