"""GPU kernels of the learned coarse step against the FP64 oracle: network
forward/loss/backward/Adam, fitting features, trace moments, and learned
parareal (with a network whose output is exact in FP32) end to end."""

import os

import numpy as np
import pytest
import torch

from oracle import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV
from oracle import mlp, learned, integrators, parareal
from paper_1505_07959_amd import inputs
from tests.gpu_util import dev, host, empty, rel, say, increments_agree

pytestmark = pytest.mark.gpu


def _f32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _net_case(S=300, seed=0):
    rng = np.random.default_rng(seed)
    theta = inputs.mlp_init(seed + 1) + 0.05 * rng.standard_normal(9288)
    theta = theta.astype(np.float32).astype(np.float64)   # exactly representable on both sides
    Xin = np.column_stack([rng.uniform(0, 1, S), rng.uniform(0.004, 0.04, S), rng.normal(size=(S, 4))])
    Xin = Xin.astype(np.float32).astype(np.float64)
    norm = np.concatenate([Xin.mean(0), Xin.std(0)]).astype(np.float32).astype(np.float64)
    return theta, Xin, norm


def test_forward_matches_oracle():
    from paper_1505_07959_amd import fm
    theta, Xin, norm = _net_case()
    Y = torch.empty((Xin.shape[0], 8), dtype=torch.float32, device="cuda")
    fm.fm_mlp_forward(_f32(theta), _f32(norm), _f32(Xin), Y)
    Z = (Xin - norm[:6]) / norm[6:]
    ref, _ = mlp.forward(theta, Z)
    e = rel(host(Y).astype(np.float64), ref)
    say("forward rel err %.2e" % e)
    assert e <= 1e-5


def test_loss_and_backward_match_oracle():
    from paper_1505_07959_amd import fm
    theta, Xin, norm = _net_case(S=257, seed=3)
    S = Xin.shape[0]
    rng = np.random.default_rng(5)
    Bm = rng.standard_normal((S, 8, 8))
    G = np.einsum("sab,scb->sac", Bm, Bm) + 0.1 * np.eye(8)
    b = rng.standard_normal((S, 8))
    f = rng.uniform(1.0, 2.0, S)
    cbase = np.tile(np.array([1.0, -1.0, 0, 0, 0.25, 0, 0, 0]), (S, 1))
    rho = 0.01
    # defect data relative to cbase, as the feature kernel writes it
    bD = b - np.einsum("sab,sb->sa", G, cbase)
    fD = f - 2 * np.einsum("sa,sa->s", b, cbase) + np.einsum("sa,sab,sb->s", cbase, G, cbase)
    Y = torch.empty((S, 8), dtype=torch.float32, device="cuda")
    acts = torch.empty((S, 192), dtype=torch.float32, device="cuda")
    dY = torch.empty((S, 8), dtype=torch.float32, device="cuda")
    Ls = torch.empty((S,), dtype=torch.float64, device="cuda")
    Lsum = torch.empty((1,), dtype=torch.float64, device="cuda")
    deltas = torch.empty((S, 192), dtype=torch.float32, device="cuda")
    grad = torch.empty((9288,), dtype=torch.float32, device="cuda")
    th, nm, xx = _f32(theta), _f32(norm), _f32(Xin)
    fm.fm_mlp_forward(th, nm, xx, Y, acts)
    fm.fm_mlp_loss(Y, _f32(cbase), dev(G.reshape(S, 64)), dev(bD), dev(fD), dev(f), rho, dY, Ls, Lsum)
    fm.fm_mlp_backward(th, nm, xx, acts, dY, deltas, grad)
    Z = (Xin - norm[:6]) / norm[6:]
    L_ref, g_ref = mlp.loss_grad(theta, Z, cbase, G, b, f, rho=rho)
    L_gpu = float(host(Lsum)[0]) / S
    say("loss %.6e vs %.6e ; grad rel err %.2e" % (L_gpu, L_ref, rel(host(grad).astype(np.float64), g_ref)))
    assert abs(L_gpu - L_ref) <= 1e-5 * abs(L_ref)
    assert rel(host(grad).astype(np.float64), g_ref) <= 1e-4


def test_adam_matches_oracle():
    from paper_1505_07959_amd import fm
    rng = np.random.default_rng(9)
    th = rng.standard_normal(9288).astype(np.float32).astype(np.float64)
    g = rng.standard_normal(9288).astype(np.float32).astype(np.float64)
    m = np.zeros(9288)
    v = np.zeros(9288)
    tt, mm, vv = _f32(th), _f32(m), _f32(v)
    for t in (1, 2, 3):
        fm.fm_mlp_adam(tt, _f32(g), mm, vv, t, 1e-3)
        th, m, v = mlp.adam_step(th, g, m, v, t, 1e-3)
    assert rel(host(tt).astype(np.float64), th) <= 1e-6


@pytest.mark.parametrize("kind", [HOMOTOPY, STEADY_INV])
def test_features_match_oracle(kind):
    from paper_1505_07959_amd import fm
    n, h = 72, 1.0 / 16
    A, Q, lam = inputs.spd(n, "loguniform", 1e-2, 10.0, 41)
    X = inputs.perturbed_identity(n, 42, 0.05)
    FX = integrators.fine(MatrixAlgebra(n), kind, A, X, h, 0.0, 4)
    G0, b0, f0 = learned.features(MatrixAlgebra(n), kind, A, X, FX, h)
    ce = learned.euler_coeffs(kind, h)
    flow = fm.fm_flow_create([(kind, dev(A))], "f64")
    try:
        G = torch.empty((3, 64), dtype=torch.float64, device="cuda")
        bD = torch.empty((3, 8), dtype=torch.float64, device="cuda")
        fD = torch.empty((3,), dtype=torch.float64, device="cuda")
        fn = torch.empty((3,), dtype=torch.float64, device="cuda")
        fm.fm_learned_features(flow, h, [dev(X)], [dev(FX)], G, bD, fD, fn, row0=1)
        mu = fm.fm_trace_moments(flow, 1)[0]
    finally:
        fm.fm_destroy(flow)
    Gg = host(G)[1].reshape(8, 8)
    assert rel(Gg, G0) <= 1e-12
    assert rel(host(bD)[1], b0 - G0 @ ce) <= 1e-9
    fD_ref = f0 - 2 * b0 @ ce + ce @ G0 @ ce
    D = FX - learned.poly_step(MatrixAlgebra(n), kind, A, X, h, ce)
    assert abs(fD_ref - np.sum(D * D)) <= 1e-6 * fD_ref     # the oracle's two routes agree
    assert abs(host(fD)[1] - np.sum(D * D)) <= 1e-9 * np.sum(D * D)
    assert abs(host(fn)[1] - f0) <= 1e-13 * f0
    assert np.allclose(mu, [np.mean((lam - 1) ** j) for j in (1, 2, 3, 4)], rtol=1e-10)


@pytest.mark.parametrize("kind,T,N,S,dtype,bar,options", [(HOMOTOPY, 1.0, 16, 8, "f64", 1e-10, None),
                                                           (STEADY_INV, 12.0, 32, 8, "f64", 1e-10, None),
                                                           (HOMOTOPY, 1.0, 16, 8, "f32", 1e-5, None),
                                                           (HOMOTOPY, 1.0, 16, 8, "f32", 1e-5, "coarse_f64=1")])
def test_learned_parareal_matches_oracle(kind, T, N, S, dtype, bar, options):
    """A network whose output is its last bias (exact in FP32): both sides use
    the same coefficients c = c_Euler(h) + b4, including the fallback choice."""
    from paper_1505_07959_amd import fm
    n = 128
    A, Q, lam = inputs.spd(n, "loguniform", 1e-2, 10.0, 51) if kind == HOMOTOPY else \
        inputs.spd(n, "loguniform", 1e-3, 1.0, 52, scale_to_unit=True)
    theta = np.zeros(9288)
    # towards the Taylor member of the homotopy step; small for the steady flow
    b4 = np.array([0.0, 0.0, 0.5, -0.5, 0.0, 0.0, 0.0, 0.0]) if kind == HOMOTOPY else \
        np.array([0.0, 0.0, 0.125, -0.03125, 0.0, 0.0, 0.0, 0.0])
    theta[-8:] = b4
    norm = np.concatenate([np.zeros(6), np.ones(6)])
    salg = SpectralAlgebra(Q, lam)
    ref = learned.parareal_learned(salg, kind, lam, salg.eye(), T, N, 1, S, 6, 0.0,
                                   lambda t, h: learned.euler_coeffs(kind, h) + b4)
    flow = fm.fm_flow_create([(kind, dev(A))], dtype, options)
    try:
        fm.fm_flow_set_coarse_model(flow, kind, theta, norm)
        out = empty(n)
        st, stats = fm.fm_parareal_solve(flow, None, [out], [{"T": T, "N": N, "fine_steps": S, "max_iter": 6,
                                                              "tol": 0.0, "coarse": fm.FM_COARSE_LEARNED}])
    finally:
        fm.fm_destroy(flow)
    e = rel(host(out), salg.to_matrix(ref["U"][-1]))
    say("learned parareal kind %d %s: iters %d, learned slices %d (oracle %d), rel err %.2e" %
        (kind, dtype, stats[0]["iters"], stats[0]["learned_slices"], sum(ref["choices"][-1]), e))
    assert stats[0]["learned_restarts"] == 0
    np.testing.assert_allclose(stats[0]["hist"], ref["increments"], rtol=1e-3 if dtype == "f32" else 1e-6)
    assert e <= bar


def test_training_pipeline_small(tmp_path):
    """Tiny end-to-end run of the training driver: samples from GPU
    trajectories, loss decreases below the Euler loss, model file round-trips
    and drives a learned parareal solve to the same fixed point as Euler.
    (The gain of a fully trained network is tested at full size.)"""
    from paper_1505_07959_amd import fm, train_coarse
    data = train_coarse.generate(HOMOTOPY, 12, 64, 1.0, [8, 16, 32], 4, 6, "f32")
    e_loss = train_coarse.euler_loss(*data[1:])
    theta, norm, hist = train_coarse.train(*data, epochs=30, minibatch=64, lr=3e-3, seed=1)
    say("euler loss %.3e, trained %.3e -> %.3e" % (e_loss, hist[0], hist[-1]))
    assert hist[-1] < 0.5 * e_loss
    path = str(tmp_path / "m.fmw")
    train_coarse.write_model(path, HOMOTOPY, theta, norm)
    k2, th2, nm2 = train_coarse.read_model(path)
    assert k2 == HOMOTOPY and np.array_equal(th2, theta) and np.array_equal(nm2, norm)
    A, Q, lam = inputs.learned_train_problem(999, 64)
    flow = fm.fm_flow_create([(HOMOTOPY, dev(A))], "f64", "coarse_model=" + path)
    try:
        out = empty(64)
        its, rs, X = {}, {}, {}
        for coarse in (fm.FM_COARSE_EULER, fm.FM_COARSE_LEARNED):
            st, stats = fm.fm_parareal_solve(flow, None, [out], [{"T": 1.0, "N": 32, "fine_steps": 8, "max_iter": 64,
                                                                  "tol": 1e-10, "coarse": coarse}])
            assert st == fm.FM_OK
            its[coarse] = stats[0]["iters"]
            rs[coarse] = stats[0]["learned_restarts"]
            X[coarse] = host(out)
        say("iterations to 1e-10: Euler %d, learned %d (restarts %d)" % (its[0], its[1], rs[1]))
        assert rel(X[fm.FM_COARSE_LEARNED], X[fm.FM_COARSE_EULER]) <= 1e-9
    finally:
        fm.fm_destroy(flow)


def _rebase_to_root_centred(theta, h):
    """A network written for the step variable K' = h A X (the fixture below
    was trained with it) re-expressed for K = h (A X - I) = K' - h I at one
    step size h: a cubic in K' is the cubic in K with coefficients
    a_i = sum_{j >= i} binom(j, i) h^(j-i) a'_j (for p and for q alike).  The
    map T is linear and maps the old Euler member (1 + h, -1, 0, ...) to the
    new one (1, -1, 0, ...), so only the output layer changes: W4 <- T W4,
    b4 <- T b4."""
    from math import comb
    Tm = np.zeros((8, 8))
    for half in (0, 4):
        for i in range(4):
            for jj in range(i, 4):
                Tm[half + i, half + jj] = comb(jj, i) * h ** (jj - i)
    th = theta.copy()
    nw4 = 8 * 64
    W4 = th[-(nw4 + 8):-8].reshape(8, 64)
    th[-(nw4 + 8):-8] = (Tm @ W4).ravel()
    th[-8:] = Tm @ th[-8:]
    return th


def test_learned_restart_matches_oracle():
    """The restart path, in a case where it happens by itself: a network
    trained for X' = X - X A X with the step variable h A X (fixture
    tests/golden/steady_k_basis_n256.fmw, trained by this project's
    train_coarse before the root-centred variable; re-expressed exactly for
    the library's K = h (A X - I), same steps), n = 256, lam ~
    loguniform[1e-3, 1], N = 32 over [0, 30], 16 RK4 steps per slice, FP64.
    Its polynomial cannot follow the flow's step at h = 30/32, the first
    sweep overflows in the oracle as on the GPU; both restart from Step 0
    with Euler, count the failed iteration, and agree on every later
    increment and on the result."""
    from paper_1505_07959_amd import fm, train_coarse
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "steady_k_basis_n256.fmw")
    kind, theta0, norm = train_coarse.read_model(path)
    n, N, S, T, K, tol = 256, 32, 16, 30.0, 32, 1e-8
    theta = _rebase_to_root_centred(theta0, T / N)
    A, Q, lam = inputs.spd(n, "loguniform", 1e-3, 1.0, 57, scale_to_unit=True)
    mu = [np.mean((lam - 1) ** j) for j in (1, 2, 3, 4)]

    def coeff(t, h):
        z = (np.array([[t, h] + mu]) - norm[:6]) / norm[6:]
        return learned.euler_coeffs(STEADY_INV, h) + mlp.forward(theta, z)[0][0]

    salg = SpectralAlgebra(Q, lam)
    with np.errstate(all="ignore"):
        ref = learned.parareal_learned(salg, STEADY_INV, lam, salg.eye(), T, N, 1, S, K, tol, coeff)
    assert ref["restarts"] == 1 and ref["status"] == "ok"
    flow = fm.fm_flow_create([(STEADY_INV, dev(A))], "f64")
    try:
        fm.fm_flow_set_coarse_model(flow, STEADY_INV, theta, norm)
        out = empty(n)
        st, stats = fm.fm_parareal_solve(flow, None, [out], [{"T": T, "N": N, "fine_steps": S, "max_iter": K,
                                                              "tol": tol, "coarse": fm.FM_COARSE_LEARNED}])
    finally:
        fm.fm_destroy(flow)
    s = stats[0]
    e = rel(host(out), salg.to_matrix(ref["U"][-1]))
    say("restart: GPU restarts %d, iters %d (oracle %d, %d), rel err %.2e" %
        (s["learned_restarts"], s["iters"], ref["restarts"], ref["iters"], e))
    assert st == fm.FM_OK and s["learned_restarts"] == 1 and s["iters"] == ref["iters"]
    increments_agree(s["hist"][1:], ref["increments"][1:])
    assert e <= 1e-10
