"""Helpers for the GPU tests: numpy <-> device tensors and a context per geometry."""
import numpy as np


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def empty_like_np(shape, dtype=np.complex128):
    import torch

    tdt = {np.complex128: torch.complex128, np.float64: torch.float64}[dtype]
    return torch.empty(shape, dtype=tdt, device="cuda")


def rel_err(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def say(*a):
    print(*a, flush=True)
