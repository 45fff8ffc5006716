"""Fine and coarse propagators (test infrastructure only).

Sec. 1 states that any explicit time marching scheme (forward Euler, Runge-Kutta)
applied to the matrix ODE approximates f(A); Alg. 1 (Sec. 2) needs a cheap
coarse propagator G(T_{n+1}, T_n, x) and an accurate fine propagator
F(T_{n+1}, T_n, x), both mapping a value at T_n to one at T_{n+1}.

* Fine F: `steps` classical four-stage Runge-Kutta steps of size
  h = (T_{n+1} - T_n) / steps:
      k1 = F(X), k2 = F(X + h/2 k1), k3 = F(X + h/2 k2), k4 = F(X + h k3),
      X <- X + h/6 (k1 + 2 k2 + 2 k3 + k4).
* Coarse G: `steps` forward-Euler steps X <- X + h F(X).
* Crank-Nicolson (Sec. 2, Example 2 computes exp(B) with Crank-Nicolson
  coarse and fine propagators), for the linear flows F(X) = s A X + b I
  (EXP: s = 1, b = 0; INV_LINEAR: s = -1, b = 1): the trapezoidal rule
  X+ - X = h/2 (F(X+) + F(X)), i.e. one linear solve per step,
      (I - s h/2 A) X+ = (I + s h/2 A) X + h b I.

The flows are autonomous, so only the step size depends on the times.

Parity: pinned by convergence order (RK4 error ratio 16, Euler ratio 2,
Crank-Nicolson ratio 4 when h halves) against the closed forms in ``exact``;
Crank-Nicolson also by its scalar form, the (1,1) Pade approximant
(1 + z/2) / (1 - z/2) of e^z, and by keeping the steady state A^{-1} of
INV_LINEAR fixed (tests/test_oracle_flows.py).
"""

from .flows import rhs, shifted
from .core import HOMOTOPY, EXP, INV_LINEAR


def rk4_step(alg, kind, X, A, h, M=None):
    if kind == HOMOTOPY and M is None:
        M = shifted(alg, A)
    k1 = rhs(alg, kind, X, A, M)
    k2 = rhs(alg, kind, X + (h / 2) * k1, A, M)
    k3 = rhs(alg, kind, X + (h / 2) * k2, A, M)
    k4 = rhs(alg, kind, X + h * k3, A, M)
    return X + (h / 6) * (k1 + 2 * k2 + 2 * k3 + k4)


def euler_step(alg, kind, X, A, h, M=None):
    return X + h * rhs(alg, kind, X, A, M)


def fine(alg, kind, A, X, t_next, t_cur, steps):
    """F(t_next, t_cur, X): `steps` RK4 steps from t_cur to t_next."""
    h = (t_next - t_cur) / steps
    M = shifted(alg, A) if kind == HOMOTOPY else None
    for _ in range(steps):
        X = rk4_step(alg, kind, X, A, h, M)
    return X


def coarse(alg, kind, A, X, t_next, t_cur, steps=1):
    """G(t_next, t_cur, X): `steps` forward-Euler steps from t_cur to t_next."""
    h = (t_next - t_cur) / steps
    M = shifted(alg, A) if kind == HOMOTOPY else None
    for _ in range(steps):
        X = euler_step(alg, kind, X, A, h, M)
    return X


def serial_fine(alg, kind, A, X0, T, N, steps):
    """The fine propagator applied slice after slice: X_{n+1} = F(T_{n+1}, T_n, X_n).

    Returns the list [X_0, ..., X_N] on the uniform grid T_n = n T / N.
    """
    out = [X0]
    for n in range(N):
        out.append(fine(alg, kind, A, out[-1], (n + 1) * T / N, n * T / N, steps))
    return out


def _linear_coeffs(kind):
    if kind == EXP:
        return 1.0, 0.0
    if kind == INV_LINEAR:
        return -1.0, 1.0
    raise ValueError("Crank-Nicolson is defined here for the linear flows only")


def cn_step(alg, kind, X, A, h):
    """One Crank-Nicolson step: solve (I - s h/2 A) X+ = (I + s h/2 A) X + h b I."""
    s, b = _linear_coeffs(kind)
    I = alg.eye()
    M = I - (s * h / 2) * A
    rhs_ = X + (s * h / 2) * alg.mul(A, X)
    if b:
        rhs_ = rhs_ + (h * b) * I
    return alg.solve(M, rhs_)


def cn(alg, kind, A, X, t_next, t_cur, steps):
    """`steps` Crank-Nicolson steps from t_cur to t_next (fine or coarse)."""
    h = (t_next - t_cur) / steps
    for _ in range(steps):
        X = cn_step(alg, kind, X, A, h)
    return X
