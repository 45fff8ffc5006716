"""Pins for the oracle's flow fields, integrators and targets (CPU only)."""

import numpy as np
import pytest

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR, KINDS
from oracle import flows, integrators, exact
from paper_1505_07959_amd import inputs


def _problem(n=6, seed=11):
    A, Q, lam = inputs.spd(n, "uniform", 0.3, 2.0, seed)
    X0 = inputs.perturbed_identity(n, seed + 1, eps=0.2)
    return A, Q, lam, X0


@pytest.mark.parametrize("kind", KINDS)
def test_closed_form_solves_flow(kind):
    """d/dt of the closed form equals the oracle's field F(X) (non-commuting X0).

    A wrong sign, dropped term or swapped operand order in flows.rhs fails here.
    """
    A, _, _, X0 = _problem()
    alg = MatrixAlgebra(A.shape[0])
    for t in (0.0, 0.3, 0.7):
        d = 1e-5
        Xp = exact.closed_form(kind, A, X0, t + d)
        Xm = exact.closed_form(kind, A, X0, t - d) if t > 0 else None
        X = exact.closed_form(kind, A, X0, t)
        if Xm is None:
            # one-sided fourth-order stencil at t = 0
            X2 = exact.closed_form(kind, A, X0, t + 2 * d)
            X3 = exact.closed_form(kind, A, X0, t + 3 * d)
            X4 = exact.closed_form(kind, A, X0, t + 4 * d)
            deriv = (-25 * X + 48 * Xp - 36 * X2 + 16 * X3 - 3 * X4) / (12 * d)
        else:
            deriv = (Xp - Xm) / (2 * d)
        F = flows.rhs(alg, kind, X, A)
        assert np.linalg.norm(deriv - F) / np.linalg.norm(F) < 1e-7


def test_closed_form_start_and_homotopy_endpoint():
    A, Q, lam, X0 = _problem()
    for kind in KINDS:
        assert np.allclose(exact.closed_form(kind, A, X0, 0.0), X0, atol=1e-13)
    # Example 1 (Sec. 2): Q(1) = A^{-1} from Q(0) = I
    n = A.shape[0]
    Q1 = exact.closed_form(HOMOTOPY, A, np.eye(n), 1.0)
    assert np.allclose(A @ Q1, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_closed_form_scalar_matches_matrix(kind):
    A, Q, lam, _ = _problem()
    n = A.shape[0]
    t = 0.8
    Xm = exact.closed_form(kind, A, np.eye(n), t)
    Xs = (Q * exact.closed_form_scalar(kind, lam, t)) @ Q.T
    assert np.linalg.norm(Xm - Xs) / np.linalg.norm(Xm) < 1e-12


@pytest.mark.parametrize("kind", KINDS)
def test_rk4_fourth_order(kind):
    """RK4 error against the closed form drops by ~16 per halving of h."""
    A, _, _, X0 = _problem()
    alg = MatrixAlgebra(A.shape[0])
    t1 = 0.5
    ref = exact.closed_form(kind, A, X0, t1)
    errs = []
    for steps in (4, 8, 16):
        X = integrators.fine(alg, kind, A, X0, t1, 0.0, steps)
        errs.append(np.linalg.norm(X - ref) / np.linalg.norm(ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.5 and 13.0 < r2 < 19.5, errs


@pytest.mark.parametrize("kind", KINDS)
def test_euler_first_order(kind):
    A, _, _, X0 = _problem()
    alg = MatrixAlgebra(A.shape[0])
    t1 = 0.5
    ref = exact.closed_form(kind, A, X0, t1)
    errs = []
    for steps in (64, 128, 256):
        X = integrators.coarse(alg, kind, A, X0, t1, 0.0, steps)
        errs.append(np.linalg.norm(X - ref) / np.linalg.norm(ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.85 < r1 < 2.15 and 1.85 < r2 < 2.15, errs


def test_rk4_single_step_scalar_by_hand():
    """One RK4 step of x' = -(lam - 1) x^2 from x = 1, worked out by hand.

    lam = 3, h = 0.1: k1 = -2, k2 = -2 (0.9)^2 = -1.62, k3 = -2 (0.919)^2 =
    -1.689122, k4 = -2 (0.8310878)^2 = -1.38141387..., step from 1.
    """
    lam = np.array([3.0])
    alg = SpectralAlgebra(np.eye(1), lam)
    x = integrators.rk4_step(alg, HOMOTOPY, np.ones(1), lam, 0.1)
    k1 = -2.0
    k2 = -2.0 * 0.9 ** 2
    k3 = -2.0 * (1 + 0.05 * k2) ** 2
    k4 = -2.0 * (1 + 0.1 * k3) ** 2
    assert abs(k2 - (-1.62)) < 1e-15 and abs(k3 - (-1.689122)) < 1e-14
    expect = 1 + 0.1 / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert abs(x[0] - expect) < 1e-15
    # the exact value 1 / (1 + 0.2) = 0.8333..., RK4 local error O(h^5)
    assert abs(x[0] - 1 / 1.2) < 1e-4


@pytest.mark.parametrize("kind", KINDS)
def test_spectral_equals_matrix(kind):
    """Spectral decoupling: symmetric A, X0 = I (fine and coarse propagators)."""
    A, Q, lam = inputs.spd(8, "uniform", 0.2, 2.0, 5)
    malg = MatrixAlgebra(8)
    salg = SpectralAlgebra(Q, lam)
    Xm = integrators.fine(malg, kind, A, np.eye(8), 0.4, 0.0, 7)
    Xs = salg.to_matrix(integrators.fine(salg, kind, lam, salg.eye(), 0.4, 0.0, 7))
    assert np.linalg.norm(Xm - Xs) / np.linalg.norm(Xm) < 1e-13
    Gm = integrators.coarse(malg, kind, A, np.eye(8), 0.4, 0.0, 3)
    Gs = salg.to_matrix(integrators.coarse(salg, kind, lam, salg.eye(), 0.4, 0.0, 3))
    assert np.linalg.norm(Gm - Gs) / np.linalg.norm(Gm) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_nonsymmetric_by_eigenvectors(kind):
    """Brute force on a tiny non-symmetric A: X0 = I keeps X a function of A, so
    X = V diag(x(mu)) V^{-1} with the scalar recursion run on the (complex)
    eigenvalues mu.  Exercises the matrix path with A != A^T."""
    n = 5
    A = inputs.nonsymmetric(n, 21, shift=1.5, spread=0.4)
    if kind == SQRT:
        A = A @ A.T + 0.5 * np.eye(n)          # SPD for the square-root flow
    mu, V = np.linalg.eig(A)
    malg = MatrixAlgebra(n)

    class CAlg:
        spectral = True
        def eye(self):
            return np.ones(n, dtype=complex)
        def mul(self, X, Y):
            return X * Y
    Xm = integrators.fine(malg, kind, A, np.eye(n), 0.6, 0.0, 5)
    xs = integrators.fine(CAlg(), kind, mu.astype(complex), np.ones(n, complex), 0.6, 0.0, 5)
    Xs = (V * xs) @ np.linalg.inv(V)
    assert np.abs(Xs.imag).max() < 1e-10
    assert np.linalg.norm(Xm - Xs.real) / np.linalg.norm(Xm) < 1e-12


def test_targets_defining_identities():
    A, Q, lam = inputs.spd(7, "loguniform", 1e-2, 10.0, 9)
    Ainv = exact.inverse_lu(A)
    assert np.linalg.norm(A @ Ainv - np.eye(7)) < 1e-12
    S = exact.sqrt_eig(A)
    assert np.linalg.norm(S @ S - A) / np.linalg.norm(A) < 1e-14
    assert np.allclose(S, S.T, atol=1e-14) and np.linalg.eigvalsh(S).min() > 0
    assert np.allclose(np.sort(np.linalg.eigvalsh(S)), np.sort(np.sqrt(lam)), rtol=1e-12)


@pytest.mark.parametrize("kind,T", [(STEADY_INV, 30.0), (SQRT, 20.0)])
def test_steady_flows_reach_target(kind, T):
    """The stable roots: X(t) -> A^{-1} (X - XAX) and A^{1/2} (A - X^2) from X0 = I."""
    A, Q, lam = inputs.spd(6, "uniform", 0.5, 2.0, 3)
    X = exact.closed_form(kind, A, np.eye(6), T)
    assert exact.rel_fro(X, exact.target(kind, A)) < 1e-6


# ---- the linear flows (Sec. 2 Example 2; Sec. 4 Example 5)

def _taylor4(Z):
    """I + Z + Z^2/2 + Z^3/6 + Z^4/24."""
    n = Z.shape[0]
    out, term = np.eye(n), np.eye(n)
    for j in range(1, 5):
        term = term @ Z / j
        out = out + term
    return out


def test_rk4_on_linear_fields_is_the_taylor_polynomial():
    """Classical RK4 applied to X' = L(X) with L linear reproduces the
    degree-4 Taylor polynomial of the exact step: X+ = P4(hA) X for X' = A X,
    and X+ = A^{-1} + P4(-hA)(X - A^{-1}) for the affine X' = I - A X.  A
    non-symmetric A and a start not commuting with it."""
    n, h = 5, 0.3
    A = inputs.nonsymmetric(n, 7, shift=1.5, spread=0.4)
    X = inputs.perturbed_identity(n, 8, eps=0.3) + 0.2 * inputs.nonsymmetric(n, 9, shift=0.0, spread=1.0)
    alg = MatrixAlgebra(n)
    got = integrators.rk4_step(alg, EXP, X, A, h)
    assert np.linalg.norm(got - _taylor4(h * A) @ X) <= 1e-14 * np.linalg.norm(got)
    Ai = np.linalg.inv(A)
    got = integrators.rk4_step(alg, INV_LINEAR, X, A, h)
    want = Ai + _taylor4(-h * A) @ (X - Ai)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    # forward Euler is the degree-1 polynomial
    got = integrators.euler_step(alg, EXP, X, A, h)
    assert np.linalg.norm(got - (X + h * A @ X)) <= 1e-15 * np.linalg.norm(got)


def test_expm_pins():
    """exp by the library routine against independent facts: the eigenvalue
    form for symmetric A, exp(A) exp(-A) = I, and the rotation generator."""
    A, Q, lam = inputs.spd(6, "uniform", -1.0, 2.0, 3)
    E = exact.expm(A)
    assert np.linalg.norm(E - (Q * np.exp(lam)) @ Q.T) <= 1e-13 * np.linalg.norm(E)
    B = inputs.nonsymmetric(6, 4, shift=0.0, spread=1.0)
    assert np.linalg.norm(exact.expm(B) @ exact.expm(-B) - np.eye(6)) < 1e-12
    th = 0.7
    R = exact.expm(np.array([[0.0, -th], [th, 0.0]]))
    assert np.allclose(R, [[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]], atol=1e-15)


def test_linear_inverse_flow_reaches_the_inverse():
    """X' = I - A X from X0 = 0 tends to A^{-1} (Example 5); the closed form at
    large t and many Euler steps both get there."""
    A, Q, lam = inputs.spd(6, "uniform", 0.5, 2.0, 12)
    Ai = np.linalg.inv(A)
    X = exact.closed_form(INV_LINEAR, A, np.zeros((6, 6)), 60.0)
    assert np.linalg.norm(X - Ai) <= 1e-12 * np.linalg.norm(Ai)
    Xe = integrators.coarse(MatrixAlgebra(6), INV_LINEAR, A, np.zeros((6, 6)), 60.0, 0.0, 600)
    assert np.linalg.norm(Xe - Ai) <= 1e-10 * np.linalg.norm(Ai)
    assert exact.target(INV_LINEAR, A) is not None
    assert np.allclose(exact.target(EXP, A, 0.5), (Q * np.exp(0.5 * lam)) @ Q.T, atol=1e-13)


def test_laplacian_generators():
    """The stencil matrices of Examples 1 and 5 against their known spectra."""
    n = 12
    lam = np.linalg.eigvalsh(inputs.laplacian_1d(n))
    j = np.arange(1, n + 1)
    want = 4 * (n + 1) ** 2 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    assert np.allclose(lam, np.sort(want), rtol=1e-12)
    m = 5
    L2 = inputs.laplacian_2d(m)
    mu = 4 * (m + 1) ** 2 * np.sin(np.arange(1, m + 1) * np.pi / (2 * (m + 1))) ** 2
    assert np.allclose(np.linalg.eigvalsh(L2), np.sort(np.add.outer(mu, mu).ravel()), rtol=1e-12)


def test_reflector_generator():
    A, Q, lam = inputs.spd_reflector(40, 0.5, 2.0, 3)
    assert np.allclose(Q @ Q, np.eye(40), atol=1e-14)
    assert np.allclose(A, (Q * lam) @ Q, atol=1e-13) and np.array_equal(A, A.T)


# ---- Crank-Nicolson (Sec. 2, Example 2) -----------------------------------

@pytest.mark.parametrize("kind", [EXP, INV_LINEAR])
def test_crank_nicolson_second_order(kind):
    """Error against the closed form (non-commuting start) falls by 4 when h
    halves: the trapezoidal rule is second order."""
    A, _, _, X0 = _problem(6, 31)
    A = -A if kind == EXP else A
    alg = MatrixAlgebra(6)
    T = 0.8
    errs = []
    for steps in (8, 16, 32):
        X = integrators.cn(alg, kind, A, X0, T, 0.0, steps)
        errs.append(np.linalg.norm(X - exact.closed_form(kind, A, X0, T)))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


def test_crank_nicolson_is_the_pade_approximant_by_eigenvectors():
    """On a non-symmetric diagonalisable A, one step of the exponential flow
    is V diag(r(h lam)) V^{-1} X with r(z) = (1 + z/2) / (1 - z/2), the (1,1)
    Pade approximant of e^z, evaluated through a complex eigendecomposition
    (an independent route: no linear solve)."""
    n = 7
    A = inputs.nonsymmetric(n, 33, shift=-1.0, spread=0.8)
    X0 = inputs.perturbed_identity(n, 34, eps=0.3)
    alg = MatrixAlgebra(n)
    h = 0.37
    lam, V = np.linalg.eig(A)
    r = (1 + h * lam / 2) / (1 - h * lam / 2)
    ref = (V @ np.diag(r) @ np.linalg.inv(V) @ X0).real
    got = integrators.cn_step(alg, EXP, X0, A, h)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # the spectral algebra takes the same step on eigenvalues
    As, Q, lam_s = inputs.spd(n, "uniform", 0.2, 3.0, 35)
    x = integrators.cn_step(SpectralAlgebra(Q, lam_s), EXP, np.ones(n), lam_s, h)
    M = integrators.cn_step(alg, EXP, np.eye(n), As, h)
    assert np.linalg.norm((Q * x) @ Q.T - M) <= 1e-13 * np.linalg.norm(M)


def test_crank_nicolson_keeps_the_steady_state():
    """The inverse A^{-1}, steady state of dX/dt = I - A X, is a fixed point of
    every Crank-Nicolson step (the trapezoidal rule preserves equilibria of
    a linear field), whatever the step size; and a long run converges to it."""
    A, _, _, X0 = _problem(6, 36)
    alg = MatrixAlgebra(6)
    Ainv = exact.inverse_lu(A)
    for h in (0.01, 0.5, 3.0):
        X = integrators.cn_step(alg, INV_LINEAR, Ainv, A, h)
        assert np.linalg.norm(X - Ainv) <= 1e-13 * np.linalg.norm(Ainv)
    X = integrators.cn(alg, INV_LINEAR, A, X0, 60.0, 0.0, 600)
    assert np.linalg.norm(X - Ainv) <= 1e-10 * np.linalg.norm(Ainv)
