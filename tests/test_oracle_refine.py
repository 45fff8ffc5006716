"""Pins for the oracle's FP64 refinement (CPU only)."""

import numpy as np

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT
from oracle import refine, exact
from paper_1505_07959_amd import inputs


def test_newton_schulz_squares_residual():
    """I - A X+ = (I - A X)^2 exactly (up to rounding) for X+ = X + X (I - A X)."""
    A = inputs.nonsymmetric(6, 2)
    alg = MatrixAlgebra(6)
    X = exact.inverse_lu(A) + 0.01 * inputs.nonsymmetric(6, 3, shift=0.0, spread=1.0)
    R, _ = refine.residual(alg, HOMOTOPY, A, X)
    Xp = refine.refine_step(alg, HOMOTOPY, A, X, R)
    Rp, _ = refine.residual(alg, HOMOTOPY, A, Xp)
    assert np.linalg.norm(Rp - R @ R) < 1e-14


def test_newton_schulz_quadratic_to_lu():
    A, Q, lam = inputs.spd(10, "loguniform", 1e-2, 10.0, 7)
    alg = MatrixAlgebra(10)
    X = exact.inverse_lu(A) * (1 + 1e-3) + 1e-4 * np.eye(10)
    X, steps, hist = refine.refine(alg, STEADY_INV, A, X, 1e-14, 6)
    assert exact.rel_fro(X, exact.inverse_lu(A)) < 1e-12
    for a, b in zip(hist[:-2], hist[1:-1]):
        assert b < 5 * a * a + 1e-15


def test_newton_sqrt_commuting_is_heron():
    """With X a function of A, the Sylvester step is Heron's (X + X^{-1} A) / 2."""
    A, Q, lam = inputs.spd(8, "uniform", 0.5, 3.0, 8)
    alg = MatrixAlgebra(8)
    X = (Q * (np.sqrt(lam) * 1.05)) @ Q.T
    R, _ = refine.residual(alg, SQRT, A, X)
    Xp = refine.refine_step(alg, SQRT, A, X, R)
    heron = 0.5 * (X + np.linalg.solve(X, A))
    assert exact.rel_fro(Xp, heron) < 1e-13


def test_newton_sqrt_noncommuting_converges():
    A, Q, lam = inputs.spd(8, "loguniform", 1e-2, 10.0, 12)
    alg = MatrixAlgebra(8)
    S = exact.sqrt_eig(A)
    P = inputs.perturbed_identity(8, 13, eps=1e-3)
    X = 0.5 * (S @ P + (S @ P).T)      # symmetric, does not commute with A
    X, steps, hist = refine.refine(alg, SQRT, A, X, 1e-14, 6)
    assert exact.rel_fro(X, S) < 1e-12 and steps <= 4


def test_spectral_refine_matches_matrix():
    A, Q, lam = inputs.spd(9, "uniform", 0.3, 2.0, 14)
    salg = SpectralAlgebra(Q, lam)
    malg = MatrixAlgebra(9)
    x = 1.0 / lam * (1 + 0.02)
    xs, _, _ = refine.refine(salg, HOMOTOPY, lam, x, 0.0, 2)
    xm, _, _ = refine.refine(malg, HOMOTOPY, A, salg.to_matrix(x), 0.0, 2)
    assert exact.rel_fro(xm, salg.to_matrix(xs)) < 1e-13
    s0 = np.sqrt(lam) * 1.03
    ss, _, _ = refine.refine(salg, SQRT, lam, s0, 0.0, 2)
    sm, _, _ = refine.refine(malg, SQRT, A, salg.to_matrix(s0), 0.0, 2)
    assert exact.rel_fro(sm, salg.to_matrix(ss)) < 1e-12
