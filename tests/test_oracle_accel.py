"""Pins for the oracle's Alg. 8 (Sec. 4, Example 5) (CPU only)."""

import numpy as np

from oracle import accel, integrators, MatrixAlgebra, INV_LINEAR
from paper_1505_07959_amd import inputs


def test_aima_matches_closed_form():
    """The loop against X_k = X* + P^k (X0 - X*) + k dt P^(k-1) e, P = I - dt A,
    for a non-symmetric A, a non-zero start and an arbitrary e.  A dropped
    accelerator term or a wrong sign fails here."""
    n, dt = 6, 0.05
    A = inputs.nonsymmetric(n, 3, shift=1.0, spread=0.4)
    X0 = 0.3 * inputs.perturbed_identity(n, 4, eps=0.5)
    e = inputs.nonsymmetric(n, 5, shift=0.2, spread=0.5)
    for k in (0, 1, 2, 7, 40):
        X, _ = accel.aima(A, X0, e, dt, k)
        want = accel.aima_closed_form(A, X0, e, dt, k)
        assert np.linalg.norm(X - want) <= 1e-12 * np.linalg.norm(want), k


def test_aima_without_accelerator_is_euler():
    n, dt = 5, 0.1
    A, _, _ = inputs.spd(n, "uniform", 0.5, 2.0, 9)
    X, _ = accel.aima(A, np.zeros((n, n)), np.zeros((n, n)), dt, 30)
    Xe = integrators.coarse(MatrixAlgebra(n), INV_LINEAR, A, np.zeros((n, n)), 30 * dt, 0.0, 30)
    assert np.linalg.norm(X - Xe) <= 1e-14 * np.linalg.norm(Xe)


def test_exact_initial_error_accelerates():
    """With e = A^{-1} - X0 the closed form gives E_k = P^(k-1) ((1 - k dt) I -
    dt A) E_0: every mode's error passes near zero at t = k dt = 1 (the
    continuous accelerator of Example 4 reaches X* at t = 1), so at t = 1 the
    accelerated residual is far below the plain Euler one; without a cut-off
    the accelerator then drives the error up again like |1 - t|."""
    n, dt = 8, 0.1
    A, Q, lam = inputs.spd(n, "loguniform", 1e-2, 1.0, 10)
    X0 = np.zeros((n, n))
    Xs = np.linalg.inv(A)
    e = Xs - X0
    _, h_acc = accel.aima(A, X0, e, dt, 200, every=10)
    _, h_pl = accel.aima(A, X0, np.zeros_like(e), dt, 200, every=10)
    ratio = np.array(h_acc) / np.array(h_pl)
    assert ratio[0] == 1.0 and ratio[1] < 0.05          # t = 1
    assert 18.0 < ratio[-1] < 20.0                       # t = 20: |1 - t| growth
    P = np.eye(n) - dt * A
    E0 = X0 - Xs
    for k in (1, 10, 13):
        want = np.linalg.matrix_power(P, k - 1) @ ((1 - k * dt) * np.eye(n) - dt * A) @ E0
        Xk, _ = accel.aima(A, X0, e, dt, k)
        assert np.linalg.norm(Xk - Xs - want) <= 1e-12 * np.linalg.norm(E0)


def test_cut_off_accelerator():
    """Switching u off at t* = 1 (k* = 1/dt) keeps the gain: from there on the
    iteration is plain Euler from the small error reached at t = 1."""
    n, dt = 8, 0.1
    A, Q, lam = inputs.spd(n, "loguniform", 1e-2, 1.0, 10)
    X0 = np.zeros((n, n))
    e = np.linalg.inv(A) - X0
    _, h_cut = accel.aima(A, X0, e, dt, 200, every=10, accel_steps=10)
    _, h_pl = accel.aima(A, X0, np.zeros_like(e), dt, 200, every=10)
    ratio = np.array(h_cut) / np.array(h_pl)
    assert np.all(ratio[1:] < 0.05)
    X10, _ = accel.aima(A, X0, e, dt, 10)
    X30, _ = accel.aima(A, X0, e, dt, 30, accel_steps=10)
    Xe = integrators.coarse(MatrixAlgebra(n), INV_LINEAR, A, X10, 2.0, 0.0, 20)
    assert np.linalg.norm(X30 - Xe) <= 1e-14 * np.linalg.norm(Xe)
