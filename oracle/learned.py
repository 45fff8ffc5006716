"""Learned coarse propagator: step family, fitting data, parareal use.

Test infrastructure only.  The paper's Alg. 1 allows any cheap coarse
propagator G; here G is a degree-3 matrix-polynomial step whose 8 coefficients
come from a small network.  Reading used (the paper does not define this part):

* Step family.  With K = h (A - I) X (HOMOTOPY) or K = h (A X - I)
  (STEADY_INV, centred on the root: K = 0 at X = A^{-1}),
      X+ = X p(K) + q(K),  p(K) = c0 I + c1 K + c2 K^2 + c3 K^3,
                           q(K) = c4 I + c5 K + c6 K^2 + c7 K^3.
  Forward Euler is the member c = (1, -1, 0, ..., 0) for both flows.  The
  exact one-step maps are X (I + K)^{-1} (HOMOTOPY) and X (I + g K)^{-1},
  g = (1 - e^{-h}) / h (STEADY_INV); (1, -1, 1, -1, 0, ...) and
  (1, -g, g^2, -g^3, 0, ...) are their third-order truncations.  For the
  steady flow the root-centred K matters: in powers of h A X the exact map's
  expansion diverges near the root once e^h > 2, in powers of h (A X - I)
  it converges along the whole path from X0 = I for 0 < A <= I.
* Network output.  The network emits a correction added to the Euler
  coefficients, so a zero network is Euler.
* Network inputs: (t, h, mu_1, ..., mu_4), mu_j = tr((A - I)^j) / n,
  standardised with the mean/std stored beside the weights.
* Fitting data.  For a state X and its fine image F(X), the basis
  E = (X, X K, X K^2, X K^3, I, K, K^2, K^3) gives X+ = sum_a c_a E_a, and the
  relative one-step defect ||X+ - F(X)||_F^2 / ||F(X)||_F^2 equals
  (c^T G c - 2 b^T c + f) / f with G_ab = <E_a, E_b>_F, b_a = <E_a, F(X)>_F,
  f = ||F(X)||_F^2.
* Fitting objective: the defect plus rho ||(c4, .., c7)||^2, rho = 1e-6.  On
  states that are functions of A the 8 basis matrices are simultaneously
  diagonal, so an unpenalised fit can trade X-terms against K-terms and pick
  huge coefficients that match the trajectory and blow up off it; the exact
  one-step maps of both flows have the form X p(K), so the penalty on q
  costs nothing where the step is right.
* Use in parareal, with the Euler step as fallback: at iteration k, for each
  slice the learned value G_L(U^k_n) is kept if finite and if its defect
  against F(U^k_n) does not exceed Euler's; otherwise Euler is used.  The
  chosen propagator G_n serves both terms of the correction
  G_n(U^{k+1}_n) - G_n(U^k_n).  Step 0 uses the learned step unless it is not
  finite.
* Restart: if a sweep still produces a non-finite iterate while the learned
  step is in use, the problem starts over from Step 0 with the Euler step on
  every slice (plain Alg. 1 from then on).  The iteration that failed counts:
  max_iter bounds all iterations, those before the restart included, and
  the increment history keeps them in order; the exactness bound k = N
  counts from the restart.  A non-finite sweep with Euler in use, or one
  that reaches max_iter, ends the run as non-finite.

Parity: pinned by the Euler member reproducing forward Euler, by the
truncation members' fourth-order local error against the closed-form maps of
both flows, by the
Gram-form defect matching the directly computed defect, by the LS solution
matching a least-squares solve on the flattened basis, by the per-slice
choice on scalar problems whose defects have closed forms (learned better on
some slices and worse on others; a choice that flips between iterations),
and by the restart reducing to plain Euler parareal
(tests/test_oracle_learned.py).
"""

import numpy as np

from .core import HOMOTOPY, STEADY_INV
from .flows import shifted
from . import integrators


def euler_coeffs(kind, h):
    if kind not in (HOMOTOPY, STEADY_INV):
        raise ValueError("learned coarse step defined for the inverse flows only")
    c = np.zeros(8)
    c[0] = 1.0
    c[1] = -1.0
    return c


def step_operator(alg, kind, A):
    return shifted(alg, A) if kind == HOMOTOPY else A


def step_variable(alg, kind, B, X, h):
    """K = h B X (HOMOTOPY, B = A - I) or h (B X - I) (STEADY_INV, B = A)."""
    K = h * alg.mul(B, X)
    return K if kind == HOMOTOPY else K - h * alg.eye()


def poly_step(alg, kind, A, X, h, c, B=None):
    """One learned step X+ = X p(K) + q(K)."""
    if B is None:
        B = step_operator(alg, kind, A)
    I = alg.eye()
    K = step_variable(alg, kind, B, X, h)
    K2 = alg.mul(K, K)
    K3 = alg.mul(K2, K)
    P = c[0] * I + c[1] * K + c[2] * K2 + c[3] * K3
    Qp = c[4] * I + c[5] * K + c[6] * K2 + c[7] * K3
    return alg.mul(X, P) + Qp


def basis(alg, kind, A, X, h):
    B = step_operator(alg, kind, A)
    I = alg.eye()
    K = step_variable(alg, kind, B, X, h)
    K2 = alg.mul(K, K)
    K3 = alg.mul(K2, K)
    return [X, alg.mul(X, K), alg.mul(X, K2), alg.mul(X, K3), I, K, K2, K3]


def features(alg, kind, A, X, FX, h):
    """(G 8x8, b 8, f) of the relative one-step defect for state X, target FX."""
    E = basis(alg, kind, A, X, h)
    G = np.empty((8, 8))
    b = np.empty(8)
    for a in range(8):
        b[a] = alg.inner(E[a], FX)
        for c in range(8):
            G[a, c] = alg.inner(E[a], E[c])
    f = alg.inner(FX, FX)
    return G, b, f


def defect_from_features(G, b, f, c):
    return float((c @ G @ c - 2 * b @ c + f) / f)


# Weight of the penalty on the q-coefficients (c4..c7) in the fitting loss.
Q_PENALTY = 1e-6


def fit_loss(G, b, f, c, rho=Q_PENALTY):
    """Fitting objective: relative defect + rho * ||(c4, .., c7)||^2."""
    return defect_from_features(G, b, f, c) + rho * float(np.sum(c[4:] ** 2))


def ls_coeffs(G, b, f=1.0, rho=Q_PENALTY):
    """Minimiser of fit_loss: (G / f + rho D_q) c = b / f, D_q = diag(0,0,0,0,1,1,1,1).

    Solved in the least-squares sense (at X = I the basis is dependent and the
    system singular; any minimiser will do)."""
    D = np.diag([0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 1.0])
    return np.linalg.lstsq(G / f + rho * D, b / f, rcond=1e-14)[0]


def moments(alg, A):
    """mu_j = tr((A - I)^j) / n, j = 1..4."""
    M = shifted(alg, A)
    P = M
    out = []
    for _ in range(4):
        out.append(alg.trace(P) / alg.n)
        P = alg.mul(P, M)
    return np.array(out)


def coarse_learned(alg, kind, A, X, t_next, t_cur, steps, coeff_fn):
    """G with `steps` learned substeps; coeff_fn(t, h) -> 8 coefficients."""
    h = (t_next - t_cur) / steps
    B = step_operator(alg, kind, A)
    for j in range(steps):
        X = poly_step(alg, kind, A, X, h, coeff_fn(t_cur + j * h, h), B)
    return X


def _finite(alg, X):
    return bool(np.all(np.isfinite(X)))


def parareal_learned(alg, kind, A, u0, T, N, coarse_steps, fine_steps,
                     max_iter, tol, coeff_fn, fine=None):
    """Alg. 1 with the learned coarse step, the per-slice Euler fallback and
    the restart with Euler after a non-finite sweep.

    fine(n, x), if given, replaces the RK4 fine propagator of slice n (tests
    use it to force a non-finite sweep).  Returns the final iterates U, the
    iteration count (all iterations, across a restart), the increments, every
    iterate list, the per-slice choices of every iteration (those of the
    coarse sweep first), the number of restarts and a status ("ok",
    "max_iter" or "nonfinite")."""
    t = [n * T / N for n in range(N + 1)]

    def F(n, x):
        if fine is not None:
            return fine(n, x)
        return integrators.fine(alg, kind, A, x, t[n + 1], t[n], fine_steps)

    def GL(n, x):
        return coarse_learned(alg, kind, A, x, t[n + 1], t[n], coarse_steps, coeff_fn)

    def GE(n, x):
        return integrators.coarse(alg, kind, A, x, t[n + 1], t[n], coarse_steps)

    def step0(learned_on):
        use = [learned_on] * N
        U0 = [u0]
        for n in range(N):
            g = GL(n, U0[n]) if learned_on else GE(n, U0[n])
            if learned_on and not _finite(alg, g):
                use[n] = False
                g = GE(n, U0[n])
            U0.append(g)
        return U0, use

    learned_on = True
    U, use_learned = step0(True)
    iterates = [list(U)]
    increments = []
    choices = [list(use_learned)]
    total = 0      # iterations run, across a restart
    k = 0          # iterations since the last Step 0
    restarts = 0
    status = "ok"
    while total < max_iter and k < N:
        F_k = [F(n, U[n]) for n in range(N)]
        G_old = []
        for n in range(N):
            ge = GE(n, U[n])
            if learned_on:
                gl = GL(n, U[n])
                dl = alg.fro(gl - F_k[n]) if _finite(alg, gl) else np.inf
                de = alg.fro(ge - F_k[n])
                use_learned[n] = bool(dl <= de)
            else:
                use_learned[n] = False
            G_old.append(gl if use_learned[n] else ge)
        U_new = [u0]
        for n in range(N):
            g_new = GL(n, U_new[n]) if use_learned[n] else GE(n, U_new[n])
            U_new.append(F_k[n] + (g_new - G_old[n]))
        inc = 0.0
        for n in range(1, N + 1):
            d = alg.fro(U_new[n] - U[n])
            s = alg.fro(U_new[n])
            q = d / s if s > 0 else d
            inc = q if q != q else max(inc, q)
        total += 1
        k += 1
        increments.append(inc)
        choices.append(list(use_learned))
        if inc != inc or not all(_finite(alg, x) for x in U_new):
            if learned_on and total < max_iter:
                learned_on = False
                restarts += 1
                k = 0
                U, use_learned = step0(False)
                iterates.append(list(U))
                continue
            U = U_new
            iterates.append(list(U))
            status = "nonfinite"
            break
        U = U_new
        iterates.append(list(U))
        if inc <= tol:
            break
    else:
        if 0 < max_iter <= total and k < N:
            status = "max_iter"
    return {"U": U, "iters": total, "increments": increments, "iterates": iterates,
            "choices": choices, "restarts": restarts, "status": status}
