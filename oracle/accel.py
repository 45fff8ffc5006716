"""Acceleration of convergence in time for the inverse (test infrastructure only).

Sec. 4 adds to the steady-state flow dX/dt = I - A X (Example 5) a forcing
u(t) that decays with the same dynamics, du/dt = -A u, u(0) = e, where e
approximates the initial error A^{-1} - X0.  Its forward-Euler
discretisation with a fixed step dt is Alg. 8 (AIMA):

    X_{k+1} = X_k + dt (I - A X_k + u_k),
    u_{k+1} = (I - dt A) u_k,              u_0 = e.

With P = I - dt A and X* = A^{-1} the error E_k = X_k - X* obeys
E_{k+1} = P E_k + dt P^k e, hence the closed form (derived here)

    X_k = X* + P^k (X0 - X*) + k dt P^{k-1} e,

which the tests use to pin the loop.  With e = 0 the iteration is forward
Euler on dX/dt = I - A X.

Alg. 8 applies u at every step.  The control of Example 4 is cut off at a
time t* (u = chi_[0,1](t) e^{-tA}(X* - X0) there); `accel_steps` = k* applies
u_k only for k < k* (None: always, as printed in Alg. 8).
"""

import numpy as np


def aima(A, X0, e, dt, steps, every=0, accel_steps=None):
    """Run Alg. 8 for `steps` iterations.  Returns (X_steps, hist) where hist
    lists ||I - A X_k||_F for k = 0, every, 2 every, ... (empty if every = 0)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    I = np.eye(n)
    X = np.array(X0, dtype=np.float64)
    u = np.array(e, dtype=np.float64)
    hist = []
    for k in range(steps):
        if every and k % every == 0:
            hist.append(float(np.linalg.norm(I - A @ X)))
        if accel_steps is not None and k >= accel_steps:
            X = X + dt * (I - A @ X)
        else:
            X = X + dt * (I - A @ X + u)
            u = u - dt * (A @ u)
    if every and steps % every == 0:
        hist.append(float(np.linalg.norm(I - A @ X)))
    return X, hist


def aima_closed_form(A, X0, e, dt, k):
    """X_k of Alg. 8 from the closed form in the module docstring."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Xs = np.linalg.solve(A, np.eye(n))
    P = np.eye(n) - dt * A
    Pk1 = np.linalg.matrix_power(P, k - 1) if k >= 1 else None
    out = Xs + np.linalg.matrix_power(P, k) @ (np.asarray(X0) - Xs)
    if k >= 1:
        out = out + k * dt * Pk1 @ np.asarray(e)
    return out
