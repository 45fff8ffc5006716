"""FP64 residuals and refinement steps (test infrastructure only).

The paper obtains f(A) from the time integration alone.  The library adds an
FP64 residual and Newton-type refinement after low-precision parareal; these
are the textbook iterations, written here as the reference for that step:

* inverse (HOMOTOPY and STEADY_INV): R = I - A X, Newton-Schulz
  X+ = X + X R, for which I - A X+ = (I - A X)^2 exactly.
  Residual reported: ||I - A X||_F / ||I||_F.
* square root (SQRT): R = A - X^2; full Newton step X+ = X + H with H solving
  the Sylvester equation X H + H X = R (Bartels-Stewart via scipy here).  When X
  commutes with A this reduces to Heron's step X+ = (X + X^{-1} A) / 2.
  Residual reported: ||A - X^2||_F / ||A||_F.

Refinement loop: compute the residual; stop if it is <= tol or `max_steps`
updates were made; otherwise update and repeat.

Parity: pinned by the exact squaring identity of Newton-Schulz, by the Heron
reduction in the commuting case and by quadratic convergence to the targets of
``exact`` (tests/test_oracle_refine.py).
"""

import numpy as np

from .core import HOMOTOPY, STEADY_INV, SQRT, INV_LINEAR


def residual(alg, kind, A, X):
    """(R, relative residual) for the target of `kind`."""
    if kind in (HOMOTOPY, STEADY_INV, INV_LINEAR):
        I = alg.eye()
        R = I - alg.mul(A, X)
        return R, alg.fro(R) / alg.fro(I)
    if kind == SQRT:
        R = A - alg.mul(X, X)
        return R, alg.fro(R) / alg.fro(A)
    raise ValueError(kind)


def solve_sylvester_sym(alg, X, R):
    """H with X H + H X = R."""
    if alg.spectral:
        return R / (2.0 * X)
    import scipy.linalg
    return scipy.linalg.solve_sylvester(X, X, R)


def refine_step(alg, kind, A, X, R):
    if kind in (HOMOTOPY, STEADY_INV, INV_LINEAR):
        return X + alg.mul(X, R)
    if kind == SQRT:
        return X + solve_sylvester_sym(alg, X, R)
    raise ValueError(kind)


def refine(alg, kind, A, X, tol, max_steps):
    """Refine X; returns (X, steps, residual history [before, after 1, ...])."""
    R, res = residual(alg, kind, A, X)
    hist = [res]
    steps = 0
    while res > tol and steps < max_steps:
        X = refine_step(alg, kind, A, X, R)
        steps += 1
        R, res = residual(alg, kind, A, X)
        hist.append(res)
    return X, steps, hist
