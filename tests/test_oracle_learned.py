"""Pins for the oracle's learned coarse step and its fitting data (CPU only)."""

import numpy as np
import pytest

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV
from oracle import learned, integrators, parareal, exact
from paper_1505_07959_amd import inputs


@pytest.mark.parametrize("kind", [HOMOTOPY, STEADY_INV])
def test_euler_member_is_forward_euler(kind):
    A, _, _ = inputs.spd(7, "uniform", 0.2, 2.0, 3)
    X = inputs.perturbed_identity(7, 4, 0.1)
    alg = MatrixAlgebra(7)
    h = 0.07
    a = learned.poly_step(alg, kind, A, X, h, learned.euler_coeffs(kind, h))
    b = integrators.euler_step(alg, kind, X, A, h)
    assert exact.rel_fro(a, b) < 1e-15


def test_taylor_member_fourth_order_local_error():
    """(1, -1, 1, -1, 0, ...) is the degree-3 truncation of X (I + K)^{-1}, the
    exact one-step map of the homotopy flow: local error O(h^4)."""
    A, _, _ = inputs.spd(6, "uniform", 0.5, 2.0, 5)
    X = inputs.perturbed_identity(6, 6, 0.1)
    alg = MatrixAlgebra(6)
    c = np.array([1.0, -1.0, 1.0, -1.0, 0, 0, 0, 0])
    errs = []
    for h in (0.1, 0.05, 0.025):
        ex = exact.closed_form(HOMOTOPY, A, X, h)
        errs.append(np.linalg.norm(learned.poly_step(alg, HOMOTOPY, A, X, h, c) - ex))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


def test_gram_defect_equals_direct_defect_and_ls():
    A, _, _ = inputs.spd(6, "loguniform", 1e-2, 10.0, 7)
    alg = MatrixAlgebra(6)
    X = inputs.perturbed_identity(6, 8, 0.1)
    h = 1.0 / 16
    FX = integrators.fine(alg, HOMOTOPY, A, X, h, 0.0, 8)
    G, b, f = learned.features(alg, HOMOTOPY, A, X, FX, h)
    rng = np.random.default_rng(0)
    E = learned.basis(alg, HOMOTOPY, A, X, h)
    for _ in range(3):
        c = rng.standard_normal(8)
        direct = np.linalg.norm(sum(ci * Ei for ci, Ei in zip(c, E)) - FX) ** 2 / np.linalg.norm(FX) ** 2
        assert abs(learned.defect_from_features(G, b, f, c) - direct) < 1e-10 * max(1, direct)
    Bflat = np.stack([e.ravel() for e in E], axis=1)
    c_lstsq = np.linalg.lstsq(Bflat, FX.ravel(), rcond=None)[0]
    c_ls = learned.ls_coeffs(G, b, f, rho=0.0)
    d_ls = learned.defect_from_features(G, b, f, c_ls)
    d_lstsq = learned.defect_from_features(G, b, f, c_lstsq)
    assert d_ls <= d_lstsq * (1 + 1e-6) + 1e-20
    d_eul = learned.defect_from_features(G, b, f, learned.euler_coeffs(HOMOTOPY, h))
    assert d_ls <= d_eul
    # the penalised fit minimises the penalised objective: compare with a
    # least-squares solve on the flattened basis augmented by sqrt(rho) rows
    rho = 1e-6
    aug = np.vstack([Bflat / np.sqrt(f), np.sqrt(rho) * np.eye(8)[4:]])
    rhs = np.concatenate([FX.ravel() / np.sqrt(f), np.zeros(4)])
    c_aug = np.linalg.lstsq(aug, rhs, rcond=None)[0]
    c_pen = learned.ls_coeffs(G, b, f, rho)
    assert learned.fit_loss(G, b, f, c_pen, rho) <= learned.fit_loss(G, b, f, c_aug, rho) * (1 + 1e-6) + 1e-20


def test_moments_from_eigenvalues():
    A, Q, lam = inputs.spd(12, "loguniform", 1e-2, 10.0, 9)
    mu = learned.moments(MatrixAlgebra(12), A)
    expect = [np.mean((lam - 1) ** j) for j in (1, 2, 3, 4)]
    assert np.allclose(mu, expect, rtol=1e-12)
    mus = learned.moments(SpectralAlgebra(Q, lam), lam)
    assert np.allclose(mus, expect, rtol=1e-13)


def test_learned_parareal_with_euler_coefficients_is_plain_parareal():
    A, Q, lam = inputs.spd(10, "uniform", 0.1, 2.0, 10)
    alg = SpectralAlgebra(Q, lam)
    N, S = 6, 8
    t = [i / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, lam, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, HOMOTOPY, lam, x, t[i + 1], t[i], 1)
    plain = parareal.parareal(F, G, alg.eye(), N, N, 0.0, alg.fro)
    lrn = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, N, 0.0,
                                   lambda tt, h: learned.euler_coeffs(HOMOTOPY, h))
    for Up, Ul in zip(plain["iterates"], lrn["iterates"]):
        for a, b in zip(Up, Ul):
            assert alg.fro(a - b) <= 1e-14 * alg.fro(a)


def test_ls_coefficients_speed_up_parareal():
    """Per-slice least-squares coefficients fitted on the serial fine trajectory
    make parareal converge in fewer iterations than Euler (the gain the learned
    step is meant to capture)."""
    A, Q, lam = inputs.spd(256, "loguniform", 1e-2, 10.0, 15)
    alg = SpectralAlgebra(Q, lam)
    N, S, tol = 32, 8, 1e-8
    ser = integrators.serial_fine(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, S)
    table = {}
    for i in range(N):
        h = 1.0 / N
        G, b, f = learned.features(alg, HOMOTOPY, lam, ser[i], ser[i + 1], h)
        table[round(i * h, 12)] = learned.ls_coeffs(G, b, f)
    coeff = lambda tt, h: table[round(tt, 12)]
    lrn = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, N, tol, coeff)
    eul = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, N, tol,
                                   lambda tt, h: learned.euler_coeffs(HOMOTOPY, h))
    assert lrn["iters"] < eul["iters"]
