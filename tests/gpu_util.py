"""Helpers for the GPU parity tests: device transfer and error norms."""
import numpy as np


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """Norm-wise relative error ||a - b|| / ||b||."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print(msg, flush=True)
