"""Classical parareal (Sec. 2, Alg. 1) -- test infrastructure only.

Time domain [0, T] split into N slices Omega_n = (T_n, T_{n+1}), T_n = n T / N.
Coarse G(T_{n+1}, T_n, x) approximates u(T_{n+1}) given u(T_n) = x (reading of
the paper's off-by-one in the definition of G); the fine F likewise, more
accurately.

Step 0 (eq. of Step 0): U^0_0 = u0, U^0_{n+1} = G(T_{n+1}, T_n, U^0_n).
Step k+1: compute F(T_{n+1}, T_n, U^k_n) for all n (the parallel part), then
sweep sequentially
    U^{k+1}_0 = u0,
    U^{k+1}_{n+1} = G(T_{n+1}, T_n, U^{k+1}_n) + F(T_{n+1}, T_n, U^k_n)
                    - G(T_{n+1}, T_n, U^k_n).
The correction is evaluated as F + (G_new - G_old), so that where the two
coarse values are bitwise equal the result is bitwise F.

The paper gives no stopping rule (its figures plot error against k).  The
reading used here: after iteration k, the increment
    delta_k = max_n ||U^{k+1}_n - U^k_n||_F / ||U^{k+1}_n||_F
is compared with `tol`; iteration stops when delta_k <= tol, when `max_iter`
iterations have run, or when k + 1 = N (then U^{k+1} equals the serial fine
solution on every slice).

Parity: pinned against the closed form of parareal on scalar linear
propagators, U^k_n = sum_{j<=k} binom(n, j) (F - G)^j G^(n-j) u0, against the
exactness property U^k_n = F^n(u0) for n <= k, and against G = F converging in
one iteration (tests/test_oracle_parareal.py).
"""


def parareal(F, G, u0, N, max_iter, tol, norm):
    """Run Alg. 1.

    F(n, x), G(n, x): propagate x from T_n to T_{n+1}.
    norm(x): Frobenius norm.
    Returns dict with the final iterate list U (length N+1), the iteration count,
    the increment history and the list of all iterates U^0, U^1, ...
    """
    U = [u0]
    G_old = []
    for n in range(N):
        g = G(n, U[n])
        G_old.append(g)
        U.append(g)
    iterates = [list(U)]
    increments = []
    k = 0
    while k < max_iter and k < N:
        F_k = [F(n, U[n]) for n in range(N)]          # uses U^k
        U_new = [u0]
        for n in range(N):
            g_new = G(n, U_new[n])
            U_new.append(F_k[n] + (g_new - G_old[n]))
            G_old[n] = g_new
        inc = 0.0
        for n in range(1, N + 1):
            d = norm(U_new[n] - U[n])
            s = norm(U_new[n])
            inc = max(inc, d / s if s > 0 else d)
        U = U_new
        k += 1
        iterates.append(list(U))
        increments.append(inc)
        if inc <= tol:
            break
    return {"U": U, "iters": k, "increments": increments, "iterates": iterates}


def uniform_times(T, N):
    return [n * T / N for n in range(N + 1)]


def max_slice_error(Us, Xs, norm):
    """max_n ||U_n - X_n||_F / ||X_n||_F over n = 1..N (trajectory error)."""
    e = 0.0
    for u, x in zip(Us[1:], Xs[1:]):
        e = max(e, norm(u - x) / norm(x))
    return e
