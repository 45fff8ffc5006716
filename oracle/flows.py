"""Right-hand sides of the matrix flows (test infrastructure only).

* HOMOTOPY: the inverse homotopy of Sec. 2, Example 1.  With A(t) = I + t(A - I)
  (the homotopy path of Sec. 1 with X0 = I) the inverse Q(t) = A(t)^{-1}
  satisfies dQ/dt = -Q (A - I) Q = Q (I - A) Q, Q(0) = I, and Q(1) = A^{-1}.
  The introduction writes the same field as X(Id - A)X; both signs agree.
* STEADY_INV: dX/dt = X - X A X.  Its stable root is A^{-1} (the steady-state
  modelling of Sec. 1: F(X) = 0 iff X = f(A), with the differential of F at
  the root having eigenvalues of negative real part; here D F = -Id at A^{-1}).
* SQRT: dX/dt = A - X^2 for SPD A; stable root the principal square root
  (differential eigenvalues -(sqrt(lam_i) + sqrt(lam_j))).
* EXP: dQ/dt = A Q with Q(0) = I (Sec. 2, Example 2: A(t) = t A, Q(t) =
  exp(t A), Q(1) = exp(A)).
* INV_LINEAR: dX/dt = I - A X (Sec. 4, Example 5), linear, stable steady
  state A^{-1} when the eigenvalues of A have positive real part.

Association order of the products is part of the definition of the discrete
method: X (M X) for the homotopy with M = A - I, X (A X) for STEADY_INV, X X for
SQRT; the linear flows multiply A from the left.

Parity: pinned by the closed-form solutions in ``exact`` (including starting
values that do not commute with A) and by the fourth-order convergence of RK4
towards them (tests/test_oracle_flows.py).
"""

from .core import HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR


def shifted(alg, A):
    """M = A - I, the homotopy direction dA(t)/dt of Sec. 1 with X0 = I."""
    return A - alg.eye()


def rhs(alg, kind, X, A, M=None):
    """Flow field F(X) for the given kind."""
    if kind == HOMOTOPY:
        if M is None:
            M = shifted(alg, A)
        return -alg.mul(X, alg.mul(M, X))
    if kind == STEADY_INV:
        return X - alg.mul(X, alg.mul(A, X))
    if kind == SQRT:
        return A - alg.mul(X, X)
    if kind == EXP:
        return alg.mul(A, X)
    if kind == INV_LINEAR:
        return alg.eye() - alg.mul(A, X)
    raise ValueError("unknown flow kind %r" % (kind,))
