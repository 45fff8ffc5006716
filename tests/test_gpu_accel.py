"""GPU parity of Alg. 8 (Sec. 4, Example 5, fm_aima) against the oracle's loop.

Small cases: non-symmetric A with eigenvalues of positive real part, a
non-zero start and an arbitrary accelerator, with the accelerator always on,
cut off, and absent.  Full size: the 5-point Laplacian on a 63 x 63 grid
(order 3969) scaled by its Frobenius norm, X0 = 0, dt = 0.1, with the
accelerator built from the exact initial error (the paper's Fig. 7 case) and
from the inverse thresholded at 1 % of its largest entry (Fig. 6 case)."""

import numpy as np
import pytest

from oracle import accel, exact, INV_LINEAR
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say

pytestmark = pytest.mark.gpu


def _aima(A, X0, E, dt, steps, accel_steps=None, every=0, dtype="f64"):
    from paper_1505_07959_amd import fm
    n = A.shape[0]
    h = fm.fm_flow_create([(fm.FM_FLOW_INV_LINEAR, dev(A))], dtype)
    try:
        out = empty(n)
        hist = fm.fm_aima(h, None if X0 is None else [dev(X0)], None if E is None else [dev(E)], dt, steps, [out],
                          accel_steps=accel_steps, every=every)
        return host(out), (hist[0] if hist else None)
    finally:
        fm.fm_destroy(h)


@pytest.mark.parametrize("n", [64, 136])
@pytest.mark.parametrize("accel_steps", [None, 15, 0])
def test_aima_matches_oracle(n, accel_steps):
    A = inputs.nonsymmetric(n, 41, shift=1.0, spread=0.3)
    X0 = 0.2 * inputs.perturbed_identity(n, 42, eps=0.5)
    E = 0.5 * inputs.nonsymmetric(n, 43, shift=0.5, spread=0.5)
    dt, steps = 0.05, 40
    ref, rh = accel.aima(A, X0, E, dt, steps, every=5, accel_steps=accel_steps)
    X, h = _aima(A, X0, E, dt, steps, accel_steps, every=5)
    e = rel(X, ref)
    say("  n=%d accel_steps=%s: vs oracle %.2e, residual %.3e -> %.3e" % (n, accel_steps, e, h[0], h[-1]))
    assert e <= 1e-12
    np.testing.assert_allclose(h, rh, rtol=1e-10)


def test_aima_zero_inputs_and_low_precision():
    """NULL X0 and E are zero matrices (plain Euler marching from 0); FP32 and
    BF16 products stay within their rounding bars of the FP64 oracle."""
    n = 96
    A, Q, lam = inputs.spd(n, "uniform", 0.5, 2.0, 44)
    ref, _ = accel.aima(A, np.zeros((n, n)), np.zeros((n, n)), 0.1, 30)
    for dtype, bar in (("f64", 1e-13), ("f32", 1e-5), ("bf16", 2e-2)):
        X, _ = _aima(A, None, None, 0.1, 30, dtype=dtype)
        e = rel(X, ref)
        say("  %s: vs oracle %.2e" % (dtype, e))
        assert e <= bar


@pytest.mark.slow
def test_aima_laplacian_3969():
    m = 63
    L = inputs.laplacian_2d(m)
    A = L / np.linalg.norm(L)
    n = m * m
    Ainv = exact.inverse_lu(A)
    X0 = np.zeros((n, n))
    dt, steps, every = 0.1, 60, 5
    # oracle: the first two iterations at full size
    ref2, _ = accel.aima(A, X0, Ainv, dt, 2)
    X2, _ = _aima(A, X0, Ainv, dt, 2)
    e2 = rel(X2, ref2)
    say("  n=%d: two steps vs oracle %.2e" % (n, e2))
    assert e2 <= 1e-12
    _, h_plain = _aima(A, X0, None, dt, steps, every=every)
    # accelerator on until t* = 1 (the cut-off control of Example 4)
    _, h_exact = _aima(A, X0, Ainv, dt, steps, accel_steps=10, every=every)
    thr = np.where(np.abs(Ainv) >= 0.01 * np.abs(Ainv).max(), Ainv, 0.0)
    _, h_thr = _aima(A, X0, thr, dt, steps, accel_steps=10, every=every)
    r_exact = np.array(h_exact) / np.array(h_plain)
    r_thr = np.array(h_thr) / np.array(h_plain)
    say("  ratio ||AY - I|| / ||AX - I|| at t = 0, 0.5, ..., 6: exact e %s" % np.array2string(r_exact, precision=3))
    say("                                              thresholded e %s" % np.array2string(r_thr, precision=3))
    # the exact accelerator removes the error at t = 1 (closed form: factor
    # P^(k-1) ((1 - k dt) I - dt A)) and the gain stays after the cut-off;
    # the thresholded one gains less
    assert np.all(r_exact[2:] < 1e-2)
    assert np.all(r_thr[1:] < 1.0) and r_thr[2] > r_exact[2]
