"""GPU parity of fm_parareal_solve (Alg. 1) against the oracle.

Small workload: inverse homotopy, n = 64, lam ~ U[0.1, 2], N = 8 slices, one
Euler step per slice, 32 RK4 steps per slice, up to 8 iterations."""

import json
import os

import numpy as np
import pytest

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT
from oracle import integrators, parareal, exact, refine
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_homotopy.json")


def _oracle_parareal(alg, kind, A, X0, T, N, S, C, K, tol):
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, kind, A, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, kind, A, x, t[i + 1], t[i], C)
    return parareal.parareal(F, G, X0, N, K, tol, alg.fro)


def _solve(A, kind, dtype, prm, X0=None):
    from paper_1505_07959_amd import fm
    n = A.shape[0]
    h = fm.fm_flow_create([(kind, dev(A))], dtype)
    try:
        out = empty(n)
        st, stats = fm.fm_parareal_solve(h, None if X0 is None else [dev(X0)], [out], [prm])
        return st, stats[0], host(out)
    finally:
        fm.fm_destroy(h)


@pytest.mark.parametrize("K", [0, 1, 3, 8])
def test_small_workload_iterates_match_oracle(K):
    A, Q, lam = inputs.small_problem()
    say("small workload K=%d" % K)
    ref = _oracle_parareal(MatrixAlgebra(64), HOMOTOPY, A, np.eye(64), 1.0, 8, 32, 1, K, 0.0)
    st, stats, X = _solve(A, HOMOTOPY, "f64", {"T": 1.0, "N": 8, "fine_steps": 32, "max_iter": K, "tol": 0.0})
    e = rel(X, ref["U"][-1])
    say("  iters %d rel err vs oracle %.3e" % (stats["iters"], e))
    assert stats["iters"] == ref["iters"] == K
    assert e <= 1e-10
    if K:
        np.testing.assert_allclose(stats["hist"][:K], ref["increments"], rtol=1e-6)


def test_small_workload_golden_and_lu():
    """Exact termination at k = N reproduces serial RK4-256; one FP64
    Newton-Schulz step brings it to the LU inverse."""
    gold = json.load(open(GOLD))
    A, Q, lam = inputs.small_problem()
    st, stats, X = _solve(A, HOMOTOPY, "f64", {"T": 1.0, "N": 8, "fine_steps": 32, "max_iter": 8, "tol": 0.0})
    np.testing.assert_allclose(np.diag(X), gold["final_diag"], rtol=1e-10)
    lu = exact.inverse_lu(A)
    e_lu = rel(X, lu)
    say("  vs LU before refinement %.3e (oracle %.3e)" % (e_lu, gold["final_error_vs_lu"]))
    assert abs(e_lu - gold["final_error_vs_lu"]) <= 1e-3 * gold["final_error_vs_lu"]
    st, stats, Xr = _solve(A, HOMOTOPY, "f64", {"T": 1.0, "N": 8, "fine_steps": 32, "max_iter": 8, "tol": 0.0,
                                                "max_refine": 1, "refine_tol": 0.0})
    e_r = rel(Xr, lu)
    say("  vs LU after 1 Newton-Schulz step %.3e; residual %.2e -> %.2e" %
        (e_r, stats["residual_before"], stats["residual"]))
    assert stats["refine_steps"] == 1 and e_r <= 1e-10


def test_tolerance_stop_matches_oracle():
    A, Q, lam = inputs.small_problem()
    ref = _oracle_parareal(MatrixAlgebra(64), HOMOTOPY, A, np.eye(64), 1.0, 8, 32, 1, 8, 1e-5)
    st, stats, X = _solve(A, HOMOTOPY, "f64", {"T": 1.0, "N": 8, "fine_steps": 32, "max_iter": 8, "tol": 1e-5})
    assert stats["iters"] == ref["iters"] == 7
    assert rel(X, ref["U"][-1]) <= 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_exact_termination_is_bitwise_serial_fine(dtype):
    """Parareal run to k = N equals the serial fine solution computed by a
    chain of fm_fine_propagate calls on the same kernels, bit for bit."""
    from paper_1505_07959_amd import fm
    n, N, S = 130, 5, 3
    A, Q, lam = inputs.spd(n, "uniform", 0.1, 2.0, 17)
    st, stats, X = _solve(A, HOMOTOPY, dtype, {"T": 1.0, "N": N, "fine_steps": S, "max_iter": N, "tol": 0.0})
    h = fm.fm_flow_create([(HOMOTOPY, dev(A))], dtype)
    try:
        x = dev(np.eye(n))
        y = empty(n)
        for s in range(N):
            fm.fm_fine_propagate(h, (s + 1) * 1.0 / N, s * 1.0 / N, S, [x], [y])
            x, y = y, x
        ser = host(x)
    finally:
        fm.fm_destroy(h)
    assert stats["iters"] == N
    assert np.array_equal(X, ser)


@pytest.mark.parametrize("kind,T,N,S,C", [(STEADY_INV, 8.0, 8, 8, 1), (SQRT, 6.0, 12, 8, 2)])
def test_steady_flows_match_oracle(kind, T, N, S, C):
    n = 96
    A, Q, lam = inputs.spd(n, "uniform", 0.3, 2.0, 23)
    say("steady kind=%d" % kind)
    ref = _oracle_parareal(MatrixAlgebra(n), kind, A, np.eye(n), T, N, S, C, 4, 0.0)
    st, stats, X = _solve(A, kind, "f64", {"T": T, "N": N, "fine_steps": S, "coarse_steps": C, "max_iter": 4,
                                           "tol": 0.0})
    e = rel(X, ref["U"][-1])
    say("  rel err %.3e" % e)
    assert e <= 1e-10


def test_nonsymmetric_tiny_brute_force():
    """Brute force on n <= 8 with a non-symmetric A and non-identity X0."""
    n = 7
    A = inputs.nonsymmetric(n, 5, shift=1.2, spread=0.3)
    X0 = inputs.perturbed_identity(n, 6, eps=0.1)
    ref = _oracle_parareal(MatrixAlgebra(n), HOMOTOPY, A, X0, 1.0, 4, 6, 1, 2, 0.0)
    st, stats, X = _solve(A, HOMOTOPY, "f64", {"T": 1.0, "N": 4, "fine_steps": 6, "max_iter": 2, "tol": 0.0},
                          X0=X0)
    assert rel(X, ref["U"][-1]) <= 1e-13


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 1e-2), ("f16", 1e-2)])
def test_low_precision_parareal_vs_oracle(dtype, tol):
    """Mixed precision (products in dtype, FP64 state and correction) against
    the FP64 oracle of the same discrete method."""
    n = 256
    A, Q, lam = inputs.spd(n, "uniform", 0.3, 2.0, 29)
    salg = SpectralAlgebra(Q, lam)
    ref = _oracle_parareal(salg, HOMOTOPY, lam, salg.eye(), 1.0, 8, 8, 1, 3, 0.0)
    st, stats, X = _solve(A, HOMOTOPY, dtype, {"T": 1.0, "N": 8, "fine_steps": 8, "max_iter": 3, "tol": 0.0})
    e = rel(X, salg.to_matrix(ref["U"][-1]))
    say("  %s rel err %.3e" % (dtype, e))
    assert e <= tol
