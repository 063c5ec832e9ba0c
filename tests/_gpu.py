"""Helpers shared by the GPU tests (device tensors, oracle comparisons)."""
import sys

import numpy as np
import torch


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm GPU")
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
