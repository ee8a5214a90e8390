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


def oracle_map(fn, items):
    """fn over items on a pool of host threads (the oracle's C calls release
    the interpreter lock); results in input order.  At most 16 threads, the
    host share of one GPU."""
    import concurrent.futures as cf
    import os
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                         else (os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))
