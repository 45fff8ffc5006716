"""GPU parity of the propagators (fm_fine_propagate / fm_coarse_propagate)
against the FP64 oracle, element by element on the same seeded inputs.

Sizes span several tiles and a ragged tail (n = 200 is padded to 256 inside
the library: 4 x 4 tiles of 64)."""

import numpy as np
import pytest

from oracle import MatrixAlgebra, HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR, integrators
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say

pytestmark = pytest.mark.gpu

# relative Frobenius tolerance of one short propagation per dtype: FP64 to
# rounding; FP32 at the FP32 bar; BF16/FP16 at the pre-refinement bar
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2, "f16": 1e-2, "bf16x3": 1e-4}


def _case(kind, n, seed):
    A, Q, lam = inputs.spd(n, "uniform", 0.3, 2.0, seed)
    X0 = inputs.perturbed_identity(n, seed + 100, eps=0.1)
    return A, X0


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind", [HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR])
@pytest.mark.parametrize("n", [200, 64])
def test_fine_propagate_matches_oracle(dtype, kind, n):
    from paper_1505_07959_amd import fm
    say("fine_propagate dtype=%s kind=%d n=%d" % (dtype, kind, n))
    A, X0 = _case(kind, n, 7)
    t0, t1, steps = 0.1, 0.35, 6
    ref = integrators.fine(MatrixAlgebra(n), kind, A, X0, t1, t0, steps)
    h = fm.fm_flow_create([(kind, dev(A))], dtype)
    try:
        out = empty(n)
        fm.fm_fine_propagate(h, t1, t0, steps, [dev(X0)], [out])
        got = host(out)
    finally:
        fm.fm_destroy(h)
    e = rel(got, ref)
    say("  rel err %.3e" % e)
    assert e <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("kind", [HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR])
def test_coarse_propagate_matches_oracle(dtype, kind):
    from paper_1505_07959_amd import fm
    n = 136
    say("coarse_propagate dtype=%s kind=%d n=%d" % (dtype, kind, n))
    A, X0 = _case(kind, n, 9)
    t0, t1, steps = 0.0, 0.25, 3
    ref = integrators.coarse(MatrixAlgebra(n), kind, A, X0, t1, t0, steps)
    h = fm.fm_flow_create([(kind, dev(A))], dtype)
    try:
        out = empty(n)
        fm.fm_coarse_propagate(h, t1, t0, steps, fm.FM_COARSE_EULER, [dev(X0)], [out])
        got = host(out)
    finally:
        fm.fm_destroy(h)
    e = rel(got, ref)
    say("  rel err %.3e" % e)
    assert e <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind", [HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR])
def test_coarse_propagate_in_fp64_option(dtype, kind):
    """Option coarse_f64=1: the coarse step of an FP32 or 16-bit flow runs its
    products in FP64, so it meets the FP64 bar against the oracle."""
    from paper_1505_07959_amd import fm
    n = 136
    say("coarse_propagate coarse_f64 dtype=%s kind=%d n=%d" % (dtype, kind, n))
    A, X0 = _case(kind, n, 9)
    t0, t1, steps = 0.0, 0.25, 3
    ref = integrators.coarse(MatrixAlgebra(n), kind, A, X0, t1, t0, steps)
    h = fm.fm_flow_create([(kind, dev(A))], dtype, "coarse_f64=1")
    try:
        out = empty(n)
        fm.fm_coarse_propagate(h, t1, t0, steps, fm.FM_COARSE_EULER, [dev(X0)], [out])
        got = host(out)
    finally:
        fm.fm_destroy(h)
    e = rel(got, ref)
    say("  rel err %.3e" % e)
    assert e <= TOL["f64"]


def test_batched_mixed_sizes_and_kinds():
    """One flow with problems of different order and kind: every member of the
    grouped launch matches its own oracle propagation."""
    from paper_1505_07959_amd import fm
    cases = [(HOMOTOPY, 96), (SQRT, 160), (STEADY_INV, 64), (HOMOTOPY, 520), (SQRT, 32)]
    As, X0s, refs = [], [], []
    for j, (kind, n) in enumerate(cases):
        A, X0 = _case(kind, n, 30 + j)
        As.append(A)
        X0s.append(X0)
        refs.append(integrators.fine(MatrixAlgebra(n), kind, A, X0, 0.2, 0.0, 4))
    h = fm.fm_flow_create([(k, dev(A)) for (k, _), A in zip(cases, As)], "f64")
    try:
        outs = [empty(n) for _, n in cases]
        fm.fm_fine_propagate(h, 0.2, 0.0, 4, [dev(x) for x in X0s], outs)
        for (kind, n), o, r in zip(cases, outs, refs):
            e = rel(host(o), r)
            say("  kind=%d n=%d rel err %.3e" % (kind, n, e))
            assert e <= 1e-12
    finally:
        fm.fm_destroy(h)


def test_invalid_arguments_are_rejected():
    from paper_1505_07959_amd import fm
    A = dev(np.eye(8))
    with pytest.raises(fm.FmError) as ei:
        fm.fm_flow_create([(7, A)], "f64")
    assert ei.value.status == fm.FM_ERR_INVALID
    h = fm.fm_flow_create([(HOMOTOPY, A)], "f64")
    try:
        with pytest.raises(fm.FmError) as ei:
            fm.fm_fine_propagate(h, 1.0, 0.0, 0, [A], [empty(8)])
        assert ei.value.status == fm.FM_ERR_INVALID
        with pytest.raises(fm.FmError) as ei:
            fm.fm_parareal_solve(h, None, [empty(8)], [{"T": 2.0, "N": 4, "fine_steps": 2}])
        assert ei.value.status == fm.FM_ERR_INVALID
    finally:
        fm.fm_destroy(h)
