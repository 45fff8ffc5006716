"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and builds matrices; it contains none of the
method's arithmetic.  Recipe for an SPD test matrix of size n:

1. rng = numpy.random.default_rng(seed)
2. eigenvalues lam drawn first: uniform U[lo, hi] or log-uniform
   exp(U[log lo, log hi])
3. G = rng.standard_normal((n, n)); Householder QR (LAPACK geqrf via
   numpy.linalg.qr), sign fix Q <- Q diag(sign(diag R))
4. A = Q diag(lam) Q^T, symmetrised as (A + A^T) / 2

Workloads (sizes as in the benchmark configurations):
* small:     n = 64, lam ~ U[0.1, 2], seed 1
* large:     n = 4096, lam ~ U[0.05, 4], seed 2
* batched:   512 instances, instance i seeded 3000 + i: n_i uniform on
             {32, 64, ..., 512} (drawn first), lam ~ loguniform[1e-2, 10];
             even i inverse homotopy (T = 1), odd i square-root flow (T = 20)
* learned:   training matrices n = 256, lam ~ loguniform[1e-2, 10], seeds
             40000 + j; evaluation n = 2048, same law, seed 4; for the
             steady inverse flow lam ~ loguniform[1e-3, 1] scaled to max 1,
             seeds 50000 + j
* steady:    n = 8192, lam ~ loguniform[1e-3, 1], seed 5, scaled by 1 / max lam
             so that ||A||_2 <= 1
"""

import os

import numpy as np


def _eigs(rng, n, law, lo, hi):
    if law == "uniform":
        return rng.uniform(lo, hi, size=n)
    if law == "loguniform":
        return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))
    raise ValueError(law)


def _orthogonal(rng, n):
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def spd(n, law, lo, hi, seed, scale_to_unit=False):
    """(A, Q, lam) with A = Q diag(lam) Q^T (FP64, C-contiguous)."""
    rng = np.random.default_rng(seed)
    lam = _eigs(rng, n, law, lo, hi)
    if scale_to_unit:
        lam = lam / lam.max()
    Q = _orthogonal(rng, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return np.ascontiguousarray(A), Q, lam


def spd_reflector(n, lo, hi, seed):
    """(A, Q, lam) for the largest orders: A = Q diag(lam) Q with the
    Householder reflector Q = I - 2 v v^T (|v| = 1, symmetric orthogonal),
    lam ~ U[lo, hi].  A is formed in O(n^2) as diag(lam) - 2 (v w^T + w v^T)
    + 4 (v^T w) v v^T, w = lam * v; Q is returned dense (the spectral oracle
    reads rows of it)."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(lo, hi, n)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    w = lam * v
    A = -2.0 * (np.outer(v, w) + np.outer(w, v))
    A += (4.0 * float(v @ w)) * np.outer(v, v)
    A[np.diag_indices(n)] += lam
    Q = -2.0 * np.outer(v, v)
    Q[np.diag_indices(n)] += 1.0
    return np.ascontiguousarray(A), Q, lam


def _cached(name, fn):
    d = os.environ.get("FM_INPUT_CACHE")
    if not d:
        return fn()
    path = os.path.join(d, name + ".npz")
    if os.path.exists(path):
        z = np.load(path)
        return z["A"], z["Q"], z["lam"]
    A, Q, lam = fn()
    os.makedirs(d, exist_ok=True)
    np.savez(path, A=A, Q=Q, lam=lam)
    return A, Q, lam


def small_problem():
    return spd(64, "uniform", 0.1, 2.0, 1)


def large_problem(n=4096):
    return _cached("large_%d" % n, lambda: spd(n, "uniform", 0.05, 4.0, 2))


def steady_problem(n=8192):
    return _cached("steady_%d" % n,
                   lambda: spd(n, "loguniform", 1e-3, 1.0, 5, scale_to_unit=True))


def learned_eval_problem(n=2048):
    return _cached("learned_eval_%d" % n, lambda: spd(n, "loguniform", 1e-2, 10.0, 4))


def learned_train_problem(j, n=256):
    return spd(n, "loguniform", 1e-2, 10.0, 40000 + j)


def steady_train_problem(j, n=256):
    """Training matrices for the learned step of dX/dt = X - X A X."""
    return spd(n, "loguniform", 1e-3, 1.0, 50000 + j, scale_to_unit=True)


BATCHED_SIZES = tuple(range(32, 513, 32))


def batched_instance(i, max_n=512):
    """Instance i of the batched workload: (kind, T, A, Q, lam)."""
    rng = np.random.default_rng(3000 + i)
    sizes = [s for s in BATCHED_SIZES if s <= max_n]
    n = int(sizes[rng.integers(0, len(sizes))])
    lam = _eigs(rng, n, "loguniform", 1e-2, 10.0)
    Q = _orthogonal(rng, n)
    A = (Q * lam) @ Q.T
    A = np.ascontiguousarray(0.5 * (A + A.T))
    kind, T = (1, 1.0) if i % 2 == 0 else (3, 20.0)
    return kind, T, A, Q, lam


def nonsymmetric(n, seed, shift=2.0, spread=0.3):
    """Random non-symmetric, well-conditioned matrix shift*I + spread*N(0,1)/sqrt(n)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(shift * np.eye(n) + spread * rng.standard_normal((n, n)) / np.sqrt(n))


def laplacian_1d(n):
    """The 1D Laplacian of the paper's Example 1 (Sec. 2) on n interior points
    of (0, 1), Dirichlet ends: (n+1)^2 tridiag(-1, 2, -1) (the h^-2-scaled
    finite-difference matrix; eigenvalues 4 (n+1)^2 sin^2(j pi / (2(n+1))))."""
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return np.ascontiguousarray((n + 1) ** 2 * T)


def laplacian_2d(m):
    """The 5-point Laplacian on an m x m interior grid of the unit square
    (Sec. 4, Example 5), order m^2, Dirichlet boundary, h^-2 scaled."""
    T = 2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    I = np.eye(m)
    return np.ascontiguousarray((m + 1) ** 2 * (np.kron(T, I) + np.kron(I, T)))


def perturbed_identity(n, seed, eps=0.05):
    """A starting value that does not commute with A: I + eps N(0,1)/sqrt(n)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(np.eye(n) + eps * rng.standard_normal((n, n)) / np.sqrt(n))


def mlp_init(seed, sizes=(6, 64, 64, 64, 8)):
    """Initial network weights (flat FP64, layer by layer: W row-major then b).

    Hidden layers: uniform(-a, a), a = sqrt(6 / (fan_in + fan_out)); biases 0;
    output layer zero so the initial network reproduces the Euler step.
    """
    rng = np.random.default_rng(seed)
    parts = []
    L = len(sizes) - 1
    for li, (i, o) in enumerate(zip(sizes[:-1], sizes[1:])):
        if li < L - 1:
            a = np.sqrt(6.0 / (i + o))
            W = rng.uniform(-a, a, size=(o, i))
        else:
            W = np.zeros((o, i))
        parts.append(W.ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts)
