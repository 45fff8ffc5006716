"""Helpers for the GPU tests: device tensors and relative errors."""

import numpy as np
import torch


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(n):
    return torch.empty((n, n), dtype=torch.float64, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(msg):
    print(msg, flush=True)
