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


# ---- per-slice choice and restart of the learned step in parareal --------
# Scalar homotopy problems: A = (a), x' = -(a - 1) x^2, whose exact one-step
# map over a slice of length H is x -> x / (1 + K), K = H (a - 1) x.  With
# 64 RK4 steps per slice the fine propagator equals that map to ~1e-11, far
# below the defects compared here, so the defects have closed forms:
#   Euler      x (1 - K):                  exact - Euler = x K^2 / (1 + K)
#   Taylor-3   x (1 - K + K^2 - K^3):      exact - step  = -x K^4 / (1 + K)
#   Euler + d  (offset d in q):            exact - step  = x K^2 / (1 + K) - d

def _scalar(a):
    return SpectralAlgebra(np.ones((1, 1)), np.array([float(a)]))


def _euler_gap(x, K):
    return x * K * K / (1 + K)


def test_choice_follows_the_defects_slice_by_slice():
    """Taylor-3 coefficients on the first half of [0, 1] (better than Euler:
    K^4 < K^2 for 0 < K < 1) and Euler plus an offset 0.2 on the second half
    (worse: the offset exceeds twice the Euler gap, which stays below 0.1):
    every iteration chooses learned, learned, Euler, Euler, and the iterates
    are those of plain parareal with Taylor-3 on the first half and Euler plus
    the offset on the second (Step 0 takes the learned step everywhere; in
    the correction the offset cancels, so on the second half it acts as
    Euler)."""
    a, N, S = 3.0, 4, 64
    alg = _scalar(a)
    taylor = np.array([1.0, -1.0, 1.0, -1.0, 0, 0, 0, 0])
    bad = np.array([1.0, -1.0, 0, 0, 0.2, 0, 0, 0])
    coeff = lambda t, h: taylor if t < 0.5 else bad
    res = learned.parareal_learned(alg, HOMOTOPY, alg.lam, alg.eye(), 1.0, N, 1, S, N, 0.0, coeff)
    for k, ch in enumerate(res["choices"][1:]):
        U = res["iterates"][k]
        for n in range(N):
            x = float(U[n][0])
            K = 0.25 * (a - 1) * x
            assert 0 < K < 1                                # the hand derivation applies
            if n >= 2:
                assert _euler_gap(x, K) < 0.1
        assert ch == [True, True, False, False], (k, ch)
    t = [i / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, alg.lam, x, t[i + 1], t[i], S)

    def G(i, x):
        if i < 2:
            return learned.coarse_learned(alg, HOMOTOPY, alg.lam, x, t[i + 1], t[i], 1, lambda tt, h: taylor)
        return integrators.coarse(alg, HOMOTOPY, alg.lam, x, t[i + 1], t[i], 1) + 0.2

    plain = parareal.parareal(F, G, alg.eye(), N, N, 0.0, alg.fro)
    assert len(plain["iterates"]) == len(res["iterates"])
    for Up, Ul in zip(plain["iterates"], res["iterates"]):
        for u, v in zip(Up, Ul):
            assert abs(float(u[0]) - float(v[0])) <= 1e-13 * abs(float(u[0]))


def test_choice_is_taken_at_the_current_iterate():
    """Learned = Euler + offset d on every slice: chosen exactly where the
    Euler gap at U^k_n is at least d / 2.  The offset cancels in the
    correction, so the iterates are plain parareal's with G = Euler + d
    (pinned by the closed form of parareal); d is chosen so that the choice
    differs between slices, changes from one iteration to the next, and
    differs from the rule evaluated at U^{k+1}_n: a reversed inequality, a
    stale choice or a choice at the new iterate would fail."""
    a, N, S = 5.0, 8, 64
    H = 1.0 / N
    alg = _scalar(a)
    d = 0.0129
    c = np.array([1.0, -1.0, 0, 0, d, 0, 0, 0])
    res = learned.parareal_learned(alg, HOMOTOPY, alg.lam, alg.eye(), 1.0, N, 1, S, N, 0.0, lambda t, h: c)
    t = [i / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, alg.lam, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, HOMOTOPY, alg.lam, x, t[i + 1], t[i], 1) + d
    plain = parareal.parareal(F, G, alg.eye(), N, N, 0.0, alg.fro)
    for Up, Ul in zip(plain["iterates"], res["iterates"]):
        for u, v in zip(Up, Ul):
            assert abs(float(u[0]) - float(v[0])) <= 1e-13 * abs(float(u[0]))

    def rule(U):
        out = []
        for n in range(N):
            x = float(U[n][0])
            out.append(bool(_euler_gap(x, H * (a - 1) * x) >= d / 2))
        return out

    expected = [rule(res["iterates"][k]) for k in range(len(res["choices"]) - 1)]
    at_new = [rule(res["iterates"][k + 1]) for k in range(len(res["choices"]) - 1)]
    assert [ch for ch in res["choices"][1:]] == expected
    assert any(len(set(e)) == 2 for e in expected)              # differs between slices
    assert any(e1 != e2 for e1, e2 in zip(expected, expected[1:]))  # changes between iterations
    assert expected != at_new                                     # not the rule at U^{k+1}
    # margin: no iterate sits within 1e-6 of the threshold
    for k in range(len(expected)):
        for n in range(N):
            x = float(res["iterates"][k][n][0])
            assert abs(_euler_gap(x, H * (a - 1) * x) - d / 2) > 1e-6


def test_restart_after_a_nonfinite_sweep_is_plain_euler_parareal():
    """A fine propagator that fails (NaN) in the first iteration makes the
    sweep non-finite: the run restarts from Step 0 with Euler and then is
    plain Euler parareal; the failed iteration counts towards max_iter and
    stays in the increment history."""
    A, Q, lam = inputs.spd(6, "uniform", 0.2, 2.0, 21)
    alg = SpectralAlgebra(Q, lam)
    N, S, tol, K = 6, 8, 1e-12, 7
    t = [i / N for i in range(N + 1)]
    taylor = np.array([1.0, -1.0, 1.0, -1.0, 0, 0, 0, 0])
    calls = [0]

    def failing_fine(i, x):
        calls[0] += 1
        y = integrators.fine(alg, HOMOTOPY, lam, x, t[i + 1], t[i], S)
        return y * np.nan if calls[0] <= N else y

    res = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, K, tol, lambda tt, h: taylor,
                                   fine=failing_fine)
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, lam, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, HOMOTOPY, lam, x, t[i + 1], t[i], 1)
    plain = parareal.parareal(F, G, alg.eye(), N, K - 1, tol, alg.fro)
    assert res["restarts"] == 1 and res["status"] == "ok"
    assert res["iters"] == 1 + plain["iters"]
    assert np.isnan(res["increments"][0])
    assert np.allclose(res["increments"][1:], plain["increments"], rtol=1e-12, atol=0)
    assert all(not any(ch) for ch in res["choices"][2:])
    for u, v in zip(plain["U"], res["U"]):
        assert alg.fro(u - v) <= 1e-14 * alg.fro(u)
    # the same failure on the last iteration max_iter allows ends the run
    calls[0] = 0
    one = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, 1, tol, lambda tt, h: taylor,
                                   fine=failing_fine)
    assert one["status"] == "nonfinite" and one["iters"] == 1 and one["restarts"] == 0


def test_steady_truncation_member_fourth_order_local_error():
    """For X' = X - X A X with K = h (A X - I) the exact one-step map is
    X (I + g K)^{-1}, g = (1 - e^{-h}) / h (from the closed form of the flow);
    the member (1, -g, g^2, -g^3, 0, ...) is its third-order truncation: local
    error O(h^4) against the closed form, from a start away from the root."""
    A, _, _ = inputs.spd(6, "uniform", 0.3, 1.0, 25)
    X = 0.6 * inputs.perturbed_identity(6, 26, 0.1)
    alg = MatrixAlgebra(6)
    errs = []
    for h in (0.1, 0.05, 0.025):
        g = (1 - np.exp(-h)) / h
        c = np.array([1.0, -g, g * g, -g ** 3, 0, 0, 0, 0])
        ex = exact.closed_form(STEADY_INV, A, X, h)
        errs.append(np.linalg.norm(learned.poly_step(alg, STEADY_INV, A, X, h, c) - ex))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


def test_steady_step_variable_vanishes_at_the_root():
    """K = h (A X - I) is zero at X = A^{-1}: every member with c0 = 1 and
    q(0) = c4 = 0 keeps the root fixed."""
    A, _, _ = inputs.spd(5, "uniform", 0.3, 1.0, 27)
    Ainv = exact.inverse_lu(A)
    alg = MatrixAlgebra(5)
    c = np.array([1.0, -0.7, 0.3, -0.1, 0.0, 0.2, -0.05, 0.01])
    X = learned.poly_step(alg, STEADY_INV, A, Ainv, 0.9, c)
    assert np.linalg.norm(X - Ainv) <= 1e-13 * np.linalg.norm(Ainv)
