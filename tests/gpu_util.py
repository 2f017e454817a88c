"""Helpers shared by the GPU tests (device transfers and printing the case
before each GPU step)."""
import sys

import numpy as np


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device="cuda:0", dtype=dtype)


def to_np(t):
    return t.detach().to("cpu").numpy()


def cdt(mixed):
    import torch
    return torch.complex64 if mixed else torch.complex128
