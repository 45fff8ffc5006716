"""Pins for the oracle's modified parareal, globalQR and diamond product
(Sec. 3, Alg. 2-4) (CPU only)."""

import numpy as np

from oracle import MatrixAlgebra, EXP, INV_LINEAR, integrators, parareal, modified
from paper_1505_07959_amd import inputs


def _fro(x):
    return float(np.sqrt(np.sum(x * x)))


def _inner(a, b):
    return float(np.sum(a * b))


def test_diamond_properties():
    """Sec. 3 proposition: s = 1 gives A^T B; X^T <> X = ||X||_F^2; an
    F-orthonormal family has Q^T <> Q = I."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((5, 3))
    B = rng.standard_normal((5, 4))
    D = modified.diamond([A[:, [i]] for i in range(3)], [B[:, [j]] for j in range(4)], _inner)
    assert np.allclose(D, A.T @ B, atol=1e-14)
    X = rng.standard_normal((4, 4))
    assert abs(modified.diamond([X], [X], _inner)[0, 0] - np.linalg.norm(X) ** 2) < 1e-12


def test_global_qr_factorisation_and_elimination():
    """Z = Q (R (x) I): every block is reproduced from the basis; the basis is
    F-orthonormal; a block dependent on earlier ones is eliminated; the
    result equals numpy's QR of the vectorised blocks up to signs."""
    rng = np.random.default_rng(1)
    Z = [rng.standard_normal((3, 3)) for _ in range(4)]
    Z.insert(2, 2.0 * Z[0] - 0.5 * Z[1])          # dependent
    Q, R, kept = modified.global_qr(Z, _inner, _fro)
    assert kept == [True, True, False, True, True] and len(Q) == 4
    for i, z in enumerate(Z):
        assert np.linalg.norm(z - sum(R[j, i] * Q[j] for j in range(len(Q)))) < 1e-12
    assert np.allclose(modified.diamond(Q, Q, _inner), np.eye(4), atol=1e-13)
    M = np.stack([z.ravel() for z in Z if z is not Z[2]], axis=1)
    q, r = np.linalg.qr(M)
    for j in range(4):
        assert np.allclose(np.abs(q[:, j]), np.abs(Q[j].ravel()), atol=1e-12)


def _setup(kind, n=4, N=8, S=10, T=1.0):
    A = inputs.nonsymmetric(n, 5, shift=-0.5 if kind == EXP else 1.0, spread=0.6)
    alg = MatrixAlgebra(n)
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, kind, A, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, kind, A, x, t[i + 1], t[i], 1)
    X0 = inputs.perturbed_identity(n, 6, eps=0.3)
    serial = [X0]
    for i in range(N):
        serial.append(F(i, serial[-1]))
    return A, F, G, X0, serial


def test_scalar_problem_is_exact_after_one_iteration():
    """1 x 1 matrices: S^0 already spans the whole space, P = I, and one
    iteration reproduces the serial fine solution."""
    for kind in (EXP, INV_LINEAR):
        A, F, G, X0, serial = _setup(kind, n=1)
        out = modified.modified_parareal(F, G, X0, 8, 1, 0.0, _fro, _inner, affine=(kind == INV_LINEAR))
        for u, s in zip(out["U"], serial):
            assert abs(u[0, 0] - s[0, 0]) <= 1e-14 * abs(s[0, 0])


def test_exactness_and_full_space():
    """U^k_n = F^n(u0) for n <= k; once the basis spans all 16 directions of
    4 x 4 matrices the sweep is the serial fine solution."""
    for kind in (EXP, INV_LINEAR):
        A, F, G, X0, serial = _setup(kind)
        for K in (1, 2, 3):
            out = modified.modified_parareal(F, G, X0, 8, K, 0.0, _fro, _inner, affine=(kind == INV_LINEAR))
            for n in range(K + 1):
                assert _fro(out["U"][n] - serial[n]) <= 1e-12 * _fro(serial[n])
        out = modified.modified_parareal(F, G, X0, 8, 8, 0.0, _fro, _inner, affine=(kind == INV_LINEAR))
        assert out["sizes"][-1] <= 16
        full = [k for k, s in enumerate(out["sizes"]) if s == 16]
        if full:
            k = full[0] + 1
            assert max(_fro(u - s) / _fro(s) for u, s in zip(out["U"], serial)) <= 1e-11


def test_faster_than_classical():
    """The paper's observation (Sec. 3, cosine example): on a linear problem
    the modified algorithm needs fewer iterations than Alg. 1 to a tolerance."""
    A, F, G, X0, serial = _setup(EXP, n=6, N=10, S=20)
    tol = 1e-10
    cl = parareal.parareal(F, G, X0, 10, 10, tol, _fro)
    md = modified.modified_parareal(F, G, X0, 10, 10, tol, _fro, _inner)
    assert md["iters"] < cl["iters"]
    assert max(_fro(u - s) / _fro(s) for u, s in zip(md["U"], serial)) < 1e-9


def test_global_qr_stays_orthonormal_on_krylov_blocks():
    """Nearly dependent blocks (a Krylov-like sequence (I + hA)^j X0, the
    coarse iterates of Step 0): the basis is F-orthonormal to rounding and
    every block is reproduced, as the proposition after Alg. 2 states."""
    n = 24
    A = inputs.nonsymmetric(n, 61, shift=0.5, spread=0.5)
    X = inputs.perturbed_identity(n, 62, eps=0.3)
    Z = [X]
    for _ in range(8):
        Z.append(Z[-1] + 0.125 * A @ Z[-1])
    Q, R, kept = modified.global_qr(Z, _inner, _fro)
    D = modified.diamond(Q, Q, _inner)
    assert np.abs(D - np.eye(len(Q))).max() < 1e-14
    for i, z in enumerate(Z):
        rec = sum(R[j, i] * Q[j] for j in range(len(Q)))
        assert _fro(z - rec) <= 1e-7 * _fro(z) * 10


def _krylov_blocks(count=15, step=0.125):
    n = 24
    A = inputs.nonsymmetric(n, 61, shift=0.5, spread=0.5)
    Z = [inputs.perturbed_identity(n, 62, eps=0.3)]
    for _ in range(count - 1):
        Z.append(Z[-1] + step * A @ Z[-1])
    return Z


def test_global_qr_against_householder_on_nearly_dependent_blocks():
    """Independent reference: LAPACK's Householder QR of the vectorised blocks
    (numpy.linalg.qr).  Its |R_jj| / ||Z_j|| are the relative remainders rho_j
    (here from 1 down to 1e-14).  Two Gram-Schmidt passes keep the basis
    F-orthonormal to rounding at every remainder, one pass does not (loss of
    orthogonality ~ eps / rho^2); every kept direction agrees with
    Householder's within 1000 eps / rho_j (the conditioning of a nearly
    dependent block; any algorithm has it); and with the drop tolerance a
    block is kept exactly when its remainder against the blocks kept before
    it (Householder QR of those and the block) exceeds 1e-7 of its norm."""
    Z = _krylov_blocks()
    M = np.stack([z.ravel() for z in Z], axis=1)
    q, r = np.linalg.qr(M)
    rho = np.abs(np.diag(r)) / np.linalg.norm(M, axis=0)
    assert rho[0] == 1.0 or abs(rho[0] - 1.0) < 1e-15
    assert rho.min() < 1e-12 and rho[rho > 1e-7].size >= 5
    # no remainder near the tolerance (the flags below are then unambiguous)
    assert np.all(np.abs(np.log10(rho / modified.DROP_TOL)) > 0.3)
    eps = np.finfo(float).eps

    Q2, R2, kept2 = modified.global_qr(Z, _inner, _fro, drop_tol=0.0)
    assert all(kept2)
    D2 = modified.diamond(Q2, Q2, _inner)
    assert np.abs(D2 - np.eye(len(Q2))).max() < 1e-14
    Q1, _, _ = modified.global_qr(Z, _inner, _fro, drop_tol=0.0, passes=1)
    D1 = modified.diamond(Q1, Q1, _inner)
    assert np.abs(D1 - np.eye(len(Q1))).max() > 1e-6        # one pass is not enough
    for j in range(len(Z)):
        if rho[j] < 1e-11:
            continue                                         # direction is rounding there
        qj = q[:, j]
        e = min(_fro(Q2[j].ravel() - qj), _fro(Q2[j].ravel() + qj))
        assert e <= 1000 * eps / rho[j], (j, e, rho[j])
        if rho[j] > modified.DROP_TOL:
            assert e <= 1e-7

    # the drop rule on a shorter sequence whose remainders (against the
    # blocks kept before) stay clear of the tolerance: 1 .. 8e-9, one block
    # dropped between two kept ones
    Z = _krylov_blocks(9, 0.14)
    Q, R, kept = modified.global_qr(Z, _inner, _fro)
    ref, acc = [], []
    for z in Z:
        Mz = np.stack([Z[i].ravel() for i in acc] + [z.ravel()], axis=1)
        rz = np.linalg.qr(Mz, mode="r")
        rem = abs(rz[-1, -1]) / _fro(z)
        assert abs(np.log10(rem / modified.DROP_TOL)) > 0.3     # unambiguous
        ref.append(bool(rem > modified.DROP_TOL))
        if ref[-1]:
            acc.append(len(ref) - 1)
    assert kept == ref and kept[6] is False and kept[7] is True and sum(kept) == 7
    assert np.abs(modified.diamond(Q, Q, _inner) - np.eye(len(Q))).max() < 1e-14
    # every block is reproduced to within its dropped remainder
    for i, z in enumerate(Z):
        rec = sum(R[j, i] * Q[j] for j in range(len(Q)))
        assert _fro(z - rec) <= (modified.DROP_TOL if not kept[i] else 1e-13) * _fro(z)
