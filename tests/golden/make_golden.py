"""Writes the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
The paper prints no numerical values (its figures are not reproduced in the
text), so every fixture here is an oracle result on a seeded input.
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import MatrixAlgebra, HOMOTOPY, integrators, parareal, exact  # noqa: E402
from paper_1505_07959_amd import inputs  # noqa: E402


def small_homotopy():
    """n = 64 inverse homotopy, N = 8, one Euler step per slice, 32 RK4 steps
    per slice, up to 8 iterations; plus serial RK4 with 256 steps."""
    A, Q, lam = inputs.small_problem()
    alg = MatrixAlgebra(64)
    N, S, K, T = 8, 32, 8, 1.0
    t = [i * T / N for i in range(N + 1)]
    F = lambda i, x: integrators.fine(alg, HOMOTOPY, A, x, t[i + 1], t[i], S)
    G = lambda i, x: integrators.coarse(alg, HOMOTOPY, A, x, t[i + 1], t[i], 1)
    res = parareal.parareal(F, G, np.eye(64), N, K, 0.0, alg.fro)
    ser = integrators.serial_fine(alg, HOMOTOPY, A, np.eye(64), T, N, S)
    serial256 = integrators.fine(alg, HOMOTOPY, A, np.eye(64), 1.0, 0.0, 256)
    lu = exact.inverse_lu(A)
    return {
        "what": "inverse homotopy dX/dt = X(I-A)X, X(0)=I, T=1 (Sec. 2, Example 1; Alg. 1)",
        "input": "inputs.small_problem(): n=64, lam~U[0.1,2], seed 1",
        "N": N, "fine_steps": S, "coarse_steps": 1, "max_iter": K,
        "iters": res["iters"],
        "increments": res["increments"],
        "max_slice_error_vs_serial": [parareal.max_slice_error(U, ser, alg.fro) for U in res["iterates"]],
        "final_error_vs_lu": exact.rel_fro(res["U"][-1], lu),
        "serial256_error_vs_lu": exact.rel_fro(serial256, lu),
        "final_diag": np.diag(res["U"][-1]).tolist(),
        "final_row0": res["U"][-1][0].tolist(),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "small_homotopy.json"), "w") as fh:
        json.dump(small_homotopy(), fh, indent=1)
    print("wrote", os.path.join(HERE, "small_homotopy.json"))
