"""The allocation-free fine propagation (fm_fine_propagate_noalloc) against
fm_fine_propagate, through the C interface: identical results on two calls
in a row (the second on a smaller problem, so the scratch holds the first
call's data), no change in free device memory across a call, and a clear
refusal of a workspace beyond the scratch."""

import numpy as np
import pytest
import torch

from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, say

pytestmark = pytest.mark.gpu


def _pair(fm, flow, ns, t1, t0, steps):
    X = [dev(inputs.perturbed_identity(n, 300 + n, 0.2)) for n in ns]
    ref = [empty(n) for n in ns]
    out = [empty(n) for n in ns]
    fm.fm_fine_propagate(flow, t1, t0, steps, X, ref)
    fm.fm_fine_propagate_noalloc(flow, t1, t0, steps, X, out)
    torch.cuda.synchronize()
    return [host(r) for r in ref], [host(o) for o in out]


@pytest.mark.parametrize("dtype", ["f64", "f16"])
def test_noalloc_matches_fine_propagate(dtype):
    from paper_1505_07959_amd import fm
    A1 = [inputs.spd(n, "uniform", 0.3, 2.0, 310 + n)[0] for n in (300, 257)]
    A2 = inputs.spd(97, "uniform", 0.3, 2.0, 411)[0]
    f1 = fm.fm_flow_create([(fm.FM_FLOW_INV_HOMOTOPY, dev(a)) for a in A1], dtype)
    f2 = fm.fm_flow_create([(fm.FM_FLOW_INV_STEADY, dev(A2))], dtype)
    try:
        # first call: two problems of orders 300 and 257, 6 RK4 steps
        ref, out = _pair(fm, f1, (300, 257), 0.25, 0.0, 6)
        for r, o in zip(ref, out):
            assert np.array_equal(r, o)
        # second call: one smaller problem (order 97), the scratch still
        # holding the first call's intermediates
        ref, out = _pair(fm, f2, (97,), 1.0, 0.5, 5)
        assert np.array_equal(ref[0], out[0])
        # no device memory taken by a call (outputs allocated beforehand)
        X = [dev(np.eye(97))]
        Y = [empty(97)]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        fm.fm_fine_propagate_noalloc(f2, 0.5, 0.0, 3, X, Y)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        say("noalloc %s: bitwise equal to fm_fine_propagate on both calls" % dtype)
    finally:
        fm.fm_destroy(f1)
        fm.fm_destroy(f2)


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    from paper_1505_07959_amd import fm
    n = 1408                      # 40 bytes x 1408^2 = 79 MB of FP64 workspace > 64 MiB
    A = np.eye(n) * 1.5
    f = fm.fm_flow_create([(fm.FM_FLOW_INV_HOMOTOPY, dev(A))], "f64", "autotune=0")
    try:
        X = [dev(np.eye(n))]
        Y = [empty(n)]
        with pytest.raises(fm.FmError) as ei:
            fm.fm_fine_propagate_noalloc(f, 0.1, 0.0, 1, X, Y)
        assert ei.value.status == fm.FM_ERR_INVALID and "scratch" in fm.fm_last_error()
    finally:
        fm.fm_destroy(f)
