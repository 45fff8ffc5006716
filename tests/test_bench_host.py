"""Host logic of bench.py (no GPU): the oracle baseline's fields, the rule
that HBM traffic is reported only for the GEMM source it was measured on,
and the refusal of a multi-GPU run."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_reports_all_and_one_core():
    n = 64
    A = np.eye(n) * 1.5
    r = bench.cpu_baseline(A, n, fine_steps_total=100, coarse_steps_total=10, sample_steps=1)
    assert r["kind"] == "oracle" and r["unit"] == "solves/s"
    assert r["value"] > 0 and r["cores"] >= 1
    assert r["value_one_core"] is None or r["value_one_core"] > 0
    assert "one core" in r["sample"]


def test_traffic_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    import hashlib
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1505_07959_amd", "csrc", "gemm.hip"), "rb").read()).hexdigest()
    key = "gemm_f64_fine_step_n4096"
    per_item = 2.5e9
    src = {key: {"bytes_per_item": per_item, "gemm_sha256": sha}}
    good = tmp_path / "good.json"
    good.write_text(json.dumps(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.traffic_for(key, 3) == per_item * 3
    stale = dict(src)
    stale[key] = dict(src[key], gemm_sha256="0" * 64)
    bad = tmp_path / "stale.json"
    bad.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.traffic_for(key, 3) is None
    assert bench.traffic_for("no_such_kernel", 3) is None


def test_multi_gpu_run_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_timed_region_takes_whole_solves_within_the_budget():
    # more steps wanted and the next solve (as long as the last) fits: go on
    assert bench.plan_next_solve(now=200.0, solve_s=150.0, steps_done=9, steps_target=20, budget_s=450.0,
                                 reserve_s=30.0)
    # it would end past the budget once the CPU baseline's reserve is counted
    assert not bench.plan_next_solve(now=300.0, solve_s=150.0, steps_done=18, steps_target=20, budget_s=450.0,
                                     reserve_s=30.0)
    # enough steps timed
    assert not bench.plan_next_solve(now=10.0, solve_s=1.0, steps_done=20, steps_target=20, budget_s=450.0,
                                     reserve_s=0.0)


def test_solve_work_counts_live_slices():
    # iteration k re-solves slices k..N-1; the sweep of iteration k takes a
    # coarse step on slices k+1..N-1, Step 0 on all N
    fine, coarse = bench.solve_work(4096, 4, 2, 3)
    assert fine == (4 + 3 + 2) * 2
    assert coarse == 4 + (3 + 2 + 1)


def test_learned_leg_runs_only_if_it_ends_within_its_limit():
    # the benchmark's usual end of the CPU baseline (~370 s): the leg fits the
    # 540 s limit; a run whose timed region used its whole 450 s budget
    # (plus the baseline) does not start it, so the command stays under 600 s
    assert bench.plan_learned_leg(now=370.0, budget_s=540.0)
    assert not bench.plan_learned_leg(now=480.0, budget_s=540.0)
    assert bench.LEARNED_LEG_S + 450.0 + 30.0 > 540.0


@pytest.mark.skipif(not os.path.exists(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                    "paper_1505_07959_amd", "libfm.so")),
                    reason="library not built")
def test_learned_leg_reports_both_coarse_steps(monkeypatch):
    """The leg's summary carries each coarse step's iterations, time, status,
    restarts and distance from the serial fine solution, and says whether
    the learned step took fewer iterations and less time."""
    from paper_1505_07959_amd import fm, measure_rows

    def rows(it_e, s_e, it_l, s_l):
        base = {"status": 0, "restarts": 0, "rel_diff_vs_serial_fine": 1e-11, "serial_fine_seconds": 2.0}
        return [dict(base, workload="homotopy_n2048_N128_S8_f64_tol1e-08_euler", iterations=it_e, seconds=s_e),
                dict(base, workload="homotopy_n2048_N128_S8_f64_tol1e-08_learned", iterations=it_l, seconds=s_l)]

    monkeypatch.setattr(measure_rows, "learned_vs_euler", lambda kind: rows(11, 22.8, 7, 16.5))
    r = bench.learned_leg(fm)
    assert r["euler"]["iterations"] == 11 and r["learned"]["iterations"] == 7
    assert r["learned"]["seconds"] == 16.5 and r["serial_fine_seconds"] == 2.0
    assert r["learned_fewer_iterations_and_faster"]
    # fewer iterations but slower is not a win
    monkeypatch.setattr(measure_rows, "learned_vs_euler", lambda kind: rows(11, 22.8, 7, 30.0))
    assert not bench.learned_leg(fm)["learned_fewer_iterations_and_faster"]
