"""Targets f(A) and closed-form flow solutions (test infrastructure only).

Targets:
* A^{-1} by LU (numpy.linalg.solve(A, I)): the value X(1) of the homotopy flow
  (Sec. 2, Example 1) and the stable root of dX/dt = X - X A X.
* A^{1/2} = Q diag(sqrt(lam)) Q^T from a symmetric eigendecomposition: the
  stable root of dX/dt = A - X^2 for SPD A.
* exp(T A) by scipy.linalg.expm (scaling and squaring with Pade): the value
  Q(T) of the exponential flow of Sec. 2, Example 2; A^{-1} again for the
  linear flow dX/dt = I - A X of Sec. 4, Example 5.

Closed-form solutions of the three flows for an arbitrary invertible start X0
(X0 need not commute with A; derived here, not printed in the paper):
* homotopy  dX/dt = -X M X:   d(X^{-1})/dt = M, so X(t) = (X0^{-1} + t M)^{-1};
  with X0 = I this is (I + t(A - I))^{-1}, the homotopy path of Sec. 1.
* steady inverse dX/dt = X - X A X:  Z = X^{-1} obeys dZ/dt = A - Z, so
  X(t) = (A + (X0^{-1} - A) e^{-t})^{-1}.
* square root dX/dt = A - X^2 (A symmetric positive definite): X = W' W^{-1}
  with W'' = A W, W(0) = I, W'(0) = X0, i.e.
  W(t) = cosh(sqrt(A) t) + sqrt(A)^{-1} sinh(sqrt(A) t) X0,
  W'(t) = sqrt(A) sinh(sqrt(A) t) + cosh(sqrt(A) t) X0.
* exponential dQ/dt = A Q:  Q(t) = exp(t A) X0.
* linear inverse dX/dt = I - A X:  X(t) = A^{-1} + exp(-t A) (X0 - A^{-1}).

Parity: the targets are pinned by their defining identities (A X = I,
X^2 = A with X SPD); the closed forms by finite-difference derivatives matching
the flow field (tests/test_oracle_flows.py).
"""

import numpy as np

from .core import HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR


def inverse_lu(A):
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.solve(A, np.eye(A.shape[0]))


def sqrt_eig(A):
    A = np.asarray(A, dtype=np.float64)
    lam, Q = np.linalg.eigh((A + A.T) / 2)
    if lam.min() <= 0:
        raise ValueError("matrix square root needs an SPD matrix")
    return (Q * np.sqrt(lam)) @ Q.T


def expm(A):
    import scipy.linalg
    return scipy.linalg.expm(np.asarray(A, dtype=np.float64))


def _fun_sym(A, f):
    lam, Q = np.linalg.eigh((A + A.T) / 2)
    return (Q * f(lam)) @ Q.T


def closed_form(kind, A, X0, t):
    """Exact X(t) of the flow started at X0 (see module docstring)."""
    A = np.asarray(A, dtype=np.float64)
    X0 = np.asarray(X0, dtype=np.float64)
    n = A.shape[0]
    I = np.eye(n)
    if kind == HOMOTOPY:
        return np.linalg.inv(np.linalg.inv(X0) + t * (A - I))
    if kind == STEADY_INV:
        return np.linalg.inv(A + (np.linalg.inv(X0) - A) * np.exp(-t))
    if kind == SQRT:
        C = _fun_sym(A, lambda l: np.cosh(np.sqrt(l) * t))
        S_over = _fun_sym(A, lambda l: np.sinh(np.sqrt(l) * t) / np.sqrt(l))
        S_times = _fun_sym(A, lambda l: np.sinh(np.sqrt(l) * t) * np.sqrt(l))
        W = C + S_over @ X0
        Wd = S_times + C @ X0
        return Wd @ np.linalg.inv(W)
    if kind == EXP:
        return expm(t * A) @ X0
    if kind == INV_LINEAR:
        Ai = inverse_lu(A)
        return Ai + expm(-t * A) @ (X0 - Ai)
    raise ValueError(kind)


def closed_form_scalar(kind, lam, t):
    """Closed forms with X0 = I evaluated per eigenvalue (vectorised)."""
    lam = np.asarray(lam, dtype=np.float64)
    if kind == HOMOTOPY:
        return 1.0 / (1.0 + t * (lam - 1.0))
    if kind == STEADY_INV:
        return 1.0 / (lam + (1.0 - lam) * np.exp(-t))
    if kind == SQRT:
        s = np.sqrt(lam)
        th = np.tanh(s * t)
        return s * (1.0 + s * th) / (s + th)
    if kind == EXP:
        return np.exp(lam * t)
    if kind == INV_LINEAR:
        return 1.0 / lam + np.exp(-lam * t) * (1.0 - 1.0 / lam)
    raise ValueError(kind)


def target(kind, A, T=1.0):
    """f(A) reached by the flow: A^{-1} (HOMOTOPY at T = 1, STEADY_INV,
    INV_LINEAR), A^{1/2}, or exp(T A) (EXP at time T)."""
    if kind in (HOMOTOPY, STEADY_INV, INV_LINEAR):
        return inverse_lu(A)
    if kind == EXP:
        return expm(T * A)
    if kind == SQRT:
        return sqrt_eig(A)
    raise ValueError(kind)


def rel_fro(X, Y):
    """||X - Y||_F / ||Y||_F."""
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))
