"""The stored oracle fixtures still match the oracle (guards silent oracle edits)."""

import json
import os

import numpy as np

from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_small_homotopy_fixture():
    stored = json.load(open(os.path.join(HERE, "small_homotopy.json")))
    now = make_golden.small_homotopy()
    assert stored["iters"] == now["iters"] == 8
    np.testing.assert_allclose(now["increments"], stored["increments"], rtol=1e-9)
    np.testing.assert_allclose(now["final_diag"], stored["final_diag"], rtol=1e-12)
    # exact termination: after N iterations parareal equals serial fine
    assert stored["max_slice_error_vs_serial"][-1] == 0.0
    # the serial RK4 error against LU is the RK4 truncation error, not rounding
    assert 1e-9 < stored["serial256_error_vs_lu"] < 1e-7
