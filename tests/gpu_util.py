"""Helpers for the GPU parity tests: numpy <-> device tensors, error norms."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def empty_like_dev(a):
    import torch
    return torch.empty(a.shape, dtype=torch.complex128, device="cuda")


def rel_err(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def maxabs_ratio(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def note(msg):
    print(msg, flush=True)
