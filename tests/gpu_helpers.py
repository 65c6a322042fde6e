"""Shared helpers for the GPU parity tests (device memory through torch)."""
import sys

import numpy as np


def note(*a):
    """Print what names the case before a GPU step, flushed."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def padded_ld(n, multiple=4):
    return max(multiple, -(-n // multiple) * multiple)
