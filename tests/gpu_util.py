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


# pytest's capture manager (set by conftest): progress lines of the long
# tests bypass output capture, so a run shows which step it is in.
_capman = None


def say(msg):
    if _capman is not None:
        with _capman.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


def increments_agree(gpu, ref, rtol=1e-6, atol=1e-14):
    """Parareal increments are norms of differences of computed iterates:
    they agree to `rtol` relative, or to the rounding of the iterates."""
    assert len(gpu) == len(ref), (len(gpu), len(ref))
    for a, b in zip(gpu, ref):
        assert abs(a - b) <= max(rtol * abs(b), atol), (a, b)
