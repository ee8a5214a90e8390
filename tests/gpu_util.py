"""Helpers for the GPU parity tests (tensor <-> numpy limb conversions)."""
import numpy as np


def dev(x):
    import torch
    arr = np.ascontiguousarray(x, dtype=np.uint32)
    return torch.from_numpy(arr.view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def rand_limbs(g, *shape):
    return g.integers(0, 2**32, size=shape, dtype=np.uint64).astype(np.uint32)
