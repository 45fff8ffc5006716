"""Full-size parity: each workload at its real size and launch configuration,
with a bounded iteration count so every test stays well under two minutes.
Reference: the spectral FP64 oracle of the same discrete method (exact for
symmetric A with X0 = I), on sampled entries Q diag(x) Q^T[r, c], and the
exact f(A) after refinement."""

import os

import numpy as np
import pytest
import torch

from oracle import SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT, integrators, parareal
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

MODELS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1505_07959_amd", "models")


def _spectral_parareal(kind, T, Q, lam, N, S, C, K):
    alg = SpectralAlgebra(Q, lam)
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, kind, lam, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, kind, lam, x, t[i + 1], t[i], C)
    return alg, parareal.parareal(F, G, alg.eye(), N, K, 0.0, alg.fro)


def _samples(n, m=400, seed=0):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, m)
    cols = rng.integers(0, n, m)
    rows[:50] = cols[:50]          # include diagonal entries
    return rows, cols


def _solve(kind, A, dtype, prm, options=None):
    from paper_1505_07959_amd import fm
    n = A.shape[0]
    flow = fm.fm_flow_create([(kind, dev(A))], dtype, options)
    try:
        out = empty(n)
        st, stats = fm.fm_parareal_solve(flow, None, [out], [prm])
        torch.cuda.synchronize()
        return st, stats[0], out
    finally:
        fm.fm_destroy(flow)


def _sample(out, rows, cols):
    return out[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()


@pytest.mark.parametrize("dtype,bar,K", [("f64", 1e-10, 1), ("f32", 1e-5, 1)])
def test_large_homotopy_full_size(dtype, bar, K):
    """n = 4096, N = 64, 16 RK4 steps per slice (the benchmark launch), K iterations."""
    n, N, S = 4096, 64, 16
    A, Q, lam = inputs.large_problem(n)
    say("large homotopy %s K=%d" % (dtype, K))
    st, s, out = _solve(HOMOTOPY, A, dtype, {"T": 1.0, "N": N, "fine_steps": S, "max_iter": K, "tol": 0.0})
    alg, ref = _spectral_parareal(HOMOTOPY, 1.0, Q, lam, N, S, 1, K)
    rows, cols = _samples(n)
    e = rel(_sample(out, rows, cols), alg.entries(ref["U"][-1], rows, cols))
    say("  iters %d, sampled rel err %.2e, increment %.3e (oracle %.3e)" %
        (s["iters"], e, s["hist"][0], ref["increments"][0]))
    assert s["iters"] == K and e <= bar
    # the increment is a norm of differences of computed iterates: FP64 to 1e-6
    # relative, FP32 to the rounding of its products
    assert abs(s["hist"][0] - ref["increments"][0]) <= (1e-6 if dtype == "f64" else 1e-4) * ref["increments"][0]


def test_steady_fp16_full_size():
    """n = 8192 X' = X - X A X, N = 32 over [0, 30], 16 RK4 steps per slice,
    FP16 products: before refinement within the FP16 bar of the oracle's
    discrete solution; after FP64 Newton-Schulz within 1e-10 of A^{-1}."""
    n, N, S, T = 8192, 32, 16, 30.0
    A, Q, lam = inputs.steady_problem(n)
    rows, cols = _samples(n)
    st, s, out = _solve(STEADY_INV, A, "f16", {"T": T, "N": N, "fine_steps": S, "max_iter": 1, "tol": 0.0})
    alg, ref = _spectral_parareal(STEADY_INV, T, Q, lam, N, S, 1, 1)
    e_pre = rel(_sample(out, rows, cols), alg.entries(ref["U"][-1], rows, cols))
    st, s2, out2 = _solve(STEADY_INV, A, "f16", {"T": T, "N": N, "fine_steps": S, "max_iter": 1, "tol": 0.0,
                                                  "max_refine": 6, "refine_tol": 1e-13})
    e_post = rel(_sample(out2, rows, cols), alg.entries(1.0 / lam, rows, cols))
    say("steady fp16: pre-refinement %.2e, after %d Newton-Schulz steps %.2e (residual %.1e -> %.1e)" %
        (e_pre, s2["refine_steps"], e_post, s2["residual_before"], s2["residual"]))
    assert e_pre <= 1e-2
    assert e_post <= 1e-10


def test_batched_full_size():
    """All 512 batched problems (n up to 512, BF16 products, two iterations):
    every problem's iterate against its oracle, then refinement to 1e-10."""
    from paper_1505_07959_amd import fm
    cases = [inputs.batched_instance(i) for i in range(512)]
    K = 2
    prm = [{"T": T, "N": 64, "fine_steps": 8, "coarse_steps": 1 if k == HOMOTOPY else 2, "max_iter": K,
            "tol": 0.0, "max_refine": 6, "refine_tol": 1e-13} for k, T, *_ in cases]
    flow = fm.fm_flow_create([(k, dev(A)) for k, T, A, Q, lam in cases], "bf16")
    try:
        outs = [empty(c[2].shape[0]) for c in cases]
        st, stats = fm.fm_parareal_solve(flow, None, outs, prm)
        torch.cuda.synchronize()
        worst = {HOMOTOPY: 0.0, SQRT: 0.0}
        for j, (kind, T, A, Q, lam) in enumerate(cases):
            n = A.shape[0]
            rows, cols = _samples(n, 64, seed=j)
            f = 1.0 / lam if kind == HOMOTOPY else np.sqrt(lam)
            alg = SpectralAlgebra(Q, lam)
            e = rel(_sample(outs[j], rows, cols), alg.entries(f, rows, cols))
            worst[kind] = max(worst[kind], e)
            assert stats[j]["iters"] == K
        say("batched 512: worst error after refinement: inverse %.2e, root %.2e" % (worst[HOMOTOPY], worst[SQRT]))
        assert max(worst.values()) <= 1e-10
    finally:
        fm.fm_destroy(flow)


@pytest.mark.skipif(not os.path.exists(os.path.join(MODELS, "homotopy_n256.fmw")), reason="no trained model")
def test_learned_full_size():
    """n = 2048, N = 128, 8 RK4 steps per slice, FP64, learned coarse step with
    the trained network: the first two iterations agree with the oracle run
    with the same per-slice coefficients (taken from the library's network
    through the oracle's FP64 forward pass) to the FP32 network precision."""
    from paper_1505_07959_amd import fm, train_coarse
    from oracle import learned, mlp
    kind, theta, norm = train_coarse.read_model(os.path.join(MODELS, "homotopy_n256.fmw"))
    n, N, S, K = 2048, 128, 8, 2
    A, Q, lam = inputs.learned_eval_problem(n)
    st, s, out = _solve(HOMOTOPY, A, "f64", {"T": 1.0, "N": N, "fine_steps": S, "max_iter": K, "tol": 0.0,
                                              "coarse": fm.FM_COARSE_LEARNED},
                        "coarse_model=" + os.path.join(MODELS, "homotopy_n256.fmw"))
    mu = [np.mean((lam - 1) ** j) for j in (1, 2, 3, 4)]

    def coeff(t, h):
        z = (np.array([[t, h] + mu]) - norm[:6]) / norm[6:]
        return learned.euler_coeffs(HOMOTOPY, h) + mlp.forward(theta, z)[0][0]

    alg = SpectralAlgebra(Q, lam)
    ref = learned.parareal_learned(alg, HOMOTOPY, lam, alg.eye(), 1.0, N, 1, S, K, 0.0, coeff)
    rows, cols = _samples(n)
    e = rel(_sample(out, rows, cols), alg.entries(ref["U"][-1], rows, cols))
    say("learned n=2048: iters %d, sampled rel err vs oracle %.2e" % (s["iters"], e))
    assert s["learned_restarts"] == 0
    assert e <= 1e-5


def test_maximum_order_fp64():
    """The largest order the interface accepts, with a ragged tail: n = 16383
    (padded to 16384), homotopy flow, FP64, N = 2 slices of 2 RK4 steps, one
    iteration; sampled entries against the spectral oracle (A = Q diag(lam) Q
    with a Householder reflector Q, formed in O(n^2))."""
    n, N, S, K = 16383, 2, 2, 1
    A, Q, lam = inputs.spd_reflector(n, 0.3, 2.0, 77)
    say("maximum order n=%d" % n)
    st, s, out = _solve(HOMOTOPY, A, "f64", {"T": 1.0, "N": N, "fine_steps": S, "max_iter": K, "tol": 0.0})
    del A
    alg, ref = _spectral_parareal(HOMOTOPY, 1.0, Q, lam, N, S, 1, K)
    rows, cols = _samples(n)
    rows[-20:] = n - 1                      # the last row and column (next to the padding)
    cols[-10:] = n - 1
    e = rel(_sample(out, rows, cols), alg.entries(ref["U"][-1], rows, cols))
    say("  iters %d, sampled rel err %.2e" % (s["iters"], e))
    assert s["iters"] == K and e <= 1e-10
