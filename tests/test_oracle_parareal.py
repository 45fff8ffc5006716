"""Pins for the oracle's classical parareal (Alg. 1), CPU only."""

from math import comb

import numpy as np
import pytest

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT
from oracle import integrators, parareal, exact
from paper_1505_07959_amd import inputs


def _closed_form_linear(f, g, u0, n, k):
    """Known closed form of parareal for scalar linear propagators F = f, G = g
    (Gander & Vandewalle 2007): U^k_n = sum_{j<=min(k,n)} C(n,j) (f-g)^j g^(n-j) u0."""
    return sum(comb(n, j) * (f - g) ** j * g ** (n - j) for j in range(min(k, n) + 1)) * u0


def test_linear_scalar_closed_form():
    """Pins Step 0, the correction formula and its indices on u' = a u."""
    a, T, N, J = -1.3, 2.0, 9, 40
    dT = T / N
    f = (1 + a * dT / J) ** J          # fine: J Euler steps (any exact multiplier works)
    g = 1 + a * dT                     # coarse: one Euler step
    u0 = 1.7
    res = parareal.parareal(lambda n, x: f * x, lambda n, x: g * x, u0, N, N, 0.0, abs)
    assert res["iters"] == N
    for k, Uk in enumerate(res["iterates"]):
        for n in range(N + 1):
            expect = _closed_form_linear(f, g, u0, n, k)
            assert abs(Uk[n] - expect) <= 1e-13 * max(1.0, abs(expect)), (k, n)


def _c1_like(n=6, N=6):
    A, Q, lam = inputs.spd(n, "uniform", 0.1, 2.0, 1)
    return A, Q, lam


def _run(alg, kind, A, X0, T, N, S, C, K, tol):
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, kind, A, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, kind, A, x, t[i + 1], t[i], C)
    return parareal.parareal(F, G, X0, N, K, tol, alg.fro)


@pytest.mark.parametrize("kind,T", [(HOMOTOPY, 1.0), (STEADY_INV, 6.0), (SQRT, 4.0)])
def test_exactness_on_first_k_slices(kind, T):
    """U^k_n equals the serial fine solution bitwise for n <= k, and U^N is the
    serial fine solution on every slice (exact termination)."""
    A, _, _ = _c1_like()
    n = A.shape[0]
    N, S = 6, 4
    alg = MatrixAlgebra(n)
    res = _run(alg, kind, A, np.eye(n), T, N, S, 1, N, 0.0)
    ser = integrators.serial_fine(alg, kind, A, np.eye(n), T, N, S)
    assert res["iters"] == N
    for k, Uk in enumerate(res["iterates"]):
        for i in range(min(k, N) + 1):
            assert np.array_equal(Uk[i], ser[i]), (k, i)
    assert parareal.max_slice_error(res["U"], ser, alg.fro) == 0.0


def test_coarse_equal_fine_converges_in_one_iteration():
    A, _, _ = _c1_like()
    n = A.shape[0]
    alg = MatrixAlgebra(n)
    N, T = 5, 1.0
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, A, x, t[i + 1], t[i], 3)
    res = parareal.parareal(F, F, np.eye(n), N, 10, 1e-300, alg.fro)
    assert res["increments"][0] == 0.0 and res["iters"] == 1


def test_error_contracts_and_stop_rule():
    """Errors against the serial fine solution shrink with k; the run stops at
    the first increment <= tol."""
    A, Q, lam = inputs.small_problem()
    alg = SpectralAlgebra(Q, lam)
    N, S = 8, 32
    res = _run(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, S, 1, 8, 1e-6)
    ser = integrators.serial_fine(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, S)
    errs = [parareal.max_slice_error(U, ser, alg.fro) for U in res["iterates"]]
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))
    incs = res["increments"]
    assert incs[-1] <= 1e-6 and all(x > 1e-6 for x in incs[:-1])


def test_matrix_and_spectral_parareal_agree():
    A, Q, lam = inputs.spd(16, "uniform", 0.1, 2.0, 4)
    m = _run(MatrixAlgebra(16), HOMOTOPY, A, np.eye(16), 1.0, 4, 8, 1, 3, 0.0)
    salg = SpectralAlgebra(Q, lam)
    s = _run(salg, HOMOTOPY, lam, salg.eye(), 1.0, 4, 8, 1, 3, 0.0)
    for Um, Us in zip(m["iterates"], s["iterates"]):
        for a, b in zip(Um, Us):
            assert exact.rel_fro(a, salg.to_matrix(b)) < 1e-13


def test_small_workload_serial_vs_lu():
    """Serial RK4 (256 steps) on the n = 64 workload approximates A^{-1} to the
    size of the RK4 truncation error (not to rounding)."""
    A, Q, lam = inputs.small_problem()
    alg = MatrixAlgebra(64)
    X = integrators.fine(alg, HOMOTOPY, A, np.eye(64), 1.0, 0.0, 256)
    e = exact.rel_fro(X, exact.inverse_lu(A))
    assert 1e-10 < e < 1e-7
