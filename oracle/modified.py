"""Modified (subspace-enhanced) parareal for linear matrix flows (Sec. 3,
Alg. 2-4) -- test infrastructure only.

Definitions of Sec. 3:
* Frobenius inner product <A, B>_F = tr(B^T A); a family is F-orthonormal when
  it is orthonormal for it.
* The diamond product of two families A = [A_1..A_p], B = [B_1..B_l] is the
  p x l matrix A^T <> B with entries <A_i, B_j>_F.
* globalQR (Alg. 2): Gram-Schmidt of Z_1..Z_k in the Frobenius inner product,
  in the modified order of Alg. 2 (each new block is projected against every
  accepted one in turn); a block whose remaining norm r_ii vanishes is
  eliminated.  Z_i = sum_j R[j, i] Q_j.  Readings: the normalisation written
  as <Q_i, Q_1>_F = 1 is <Q_i, Q_i>_F = 1 (a garble); in floating point r_ii
  counts as zero when r_ii <= drop_tol ||Z_i||_F, drop_tol = 1e-7: the
  iterates form a Krylov-like sequence whose remainders shrink geometrically,
  and a block kept with remainder rho carries a rounding error of order
  eps / rho, so smaller remainders would make the basis (not the method's
  consistency) depend on the summation order; what they would carry goes
  through the coarse propagator instead.  The projection loop of Alg. 2 is
  run twice for every block: the proposition after Alg. 2 states that the
  result is F-orthonormal, which one Gram-Schmidt pass does not deliver in
  FP64 on these nearly dependent iterates: its loss of orthogonality grows
  like eps / r_ii^2 (measured in the pin: 3e-9 at a relative remainder of
  5e-7, 4e-6 at 1e-9), while a second pass restores it to rounding level
  (Kahan's "twice is enough" result for Gram-Schmidt with one
  reorthogonalisation, B. N. Parlett, The Symmetric Eigenvalue Problem,
  1980, Sec. 6-9; for classical Gram-Schmidt: L. Giraud, J. Langou and
  M. Rozloznik, Numer. Math. 101, 2005).  The coefficients r_ji are the sums
  of both passes.  The drop tolerance: the direction of a kept block is
  determined only to about eps ||Z_i|| / r_ii by any algorithm (the pin
  compares with Householder QR of the vectorised blocks: within
  1000 eps ||Z_i|| / r_ii, measured 1.3e-8 at r_ii = 4.6e-7 ||Z_i||); with
  1e-7 no kept direction is uncertain beyond ~1e-7, and a dropped remainder
  (<= 1e-7 of its block) passes through the coarse instead of the fine
  propagator, an error of 1e-7 times the coarse propagator's one-slice
  defect.
* Projection onto span{Q}: P Y = sum_i alpha_i Q_i with (alpha_i) = Q^T <> Y.

Alg. 3 (linear homogeneous U' = B U): Step 0 is the coarse sweep of Alg. 1.
Step k+1 enlarges S^k = span(S^{k-1} u {U^k_n, n = 0..N}) by completing the
F-orthonormal basis of S^{k-1} with globalQR, computes F(T_{n+1}, T_n, Q_j)
for the new basis blocks, and sweeps
    U^{k+1}_{n+1} = F(T_{n+1}, T_n, P U^{k+1}_n) + G(T_{n+1}, T_n, (I - P) U^{k+1}_n),
with F(P U) = sum_i alpha_i F(Q_i) by linearity.
Alg. 4 (affine, U' = B U + c): F(0), G(0) are computed first (Step -1);
F(P U) = sum_i alpha_i (F(Q_i) - F(0)) + F(0) and the update subtracts G(0).

Stopping rule as for Alg. 1 (reading): the relative increment, max_iter, or
k = N; by induction U^k_n = F^n(u0) for n <= k here too, since U^k_n lies in
S^k and is reproduced by the projection.
"""

import numpy as np

DROP_TOL = 1e-7


def diamond(As, Bs, inner):
    """A^T <> B for families As, Bs (Sec. 3 definition)."""
    return np.array([[inner(a, b) for b in Bs] for a in As])


def global_qr(Z, inner, norm, prefix=(), drop_tol=DROP_TOL, passes=2):
    """Alg. 2 on the blocks Z, continuing an F-orthonormal `prefix` (kept as
    is: the basis of S^{k-1} is completed, not recomputed).  `passes`: how
    often the projection loop runs per block (2, reading M1; 1 is Alg. 2 as
    printed, kept for the test that shows why the second pass is needed).

    Returns (Q, R, kept): Q = prefix + accepted new blocks; R[j, i] the
    coefficient of Q_j in Z_i (rows for every block of Q); kept[i] tells
    whether Z_i contributed a new block."""
    Q = list(prefix)
    coeffs = []
    kept = []
    for z in Z:
        q = z
        r = {}
        for _ in range(passes):              # reading M1: the projections twice
            for j, qj in enumerate(Q):
                c = inner(q, qj)
                r[j] = r.get(j, 0.0) + c
                q = q - c * qj
        rii = norm(q)
        nz = norm(z)
        if rii > drop_tol * nz and rii > 0:
            r[len(Q)] = rii
            Q.append(q / rii)
            kept.append(True)
        else:
            kept.append(False)
        coeffs.append(r)
    R = np.zeros((len(Q), len(Z)))
    for i, r in enumerate(coeffs):
        for j, v in r.items():
            R[j, i] = v
    return Q, R, kept


def modified_parareal(F, G, u0, N, max_iter, tol, norm, inner, affine=False, drop_tol=DROP_TOL):
    """Run Alg. 3 (affine=False) or Alg. 4 (affine=True).

    F(n, x), G(n, x): fine and coarse propagation over slice n.
    Returns dict: U (final iterates), iters, increments, basis size per
    iteration."""
    zero = 0 * u0
    F0 = [F(n, zero) for n in range(N)] if affine else None   # Step -1
    G0 = [G(n, zero) for n in range(N)] if affine else None
    U = [u0]
    for n in range(N):
        U.append(G(n, U[n]))
    Q = []
    FQ = []          # FQ[j][n] = F(n, Q_j)
    increments, sizes = [], []
    k = 0
    while k < max_iter and k < N:
        Q, _, kept = global_qr(U, inner, norm, prefix=Q, drop_tol=drop_tol)
        for q in Q[len(FQ):]:
            FQ.append([F(n, q) for n in range(N)])          # the parallel part
        sizes.append(len(Q))
        U_new = [u0]
        for n in range(N):
            x = U_new[n]
            alpha = [inner(x, q) for q in Q]
            PU = zero
            FPU = zero
            for a, q, fq in zip(alpha, Q, FQ):
                PU = PU + a * q
                FPU = FPU + a * ((fq[n] - F0[n]) if affine else fq[n])
            if affine:
                FPU = FPU + F0[n]
            GR = G(n, x - PU)
            if affine:
                GR = GR - G0[n]
            U_new.append(FPU + GR)
        inc = 0.0
        for n in range(1, N + 1):
            d = norm(U_new[n] - U[n])
            s = norm(U_new[n])
            inc = max(inc, d / s if s > 0 else d)
        U = U_new
        k += 1
        increments.append(inc)
        if inc <= tol:
            break
    return {"U": U, "iters": k, "increments": increments, "sizes": sizes}
