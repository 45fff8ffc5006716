"""Benchmark: parareal solves/s and fine-propagator MFMA TFLOP/s on one MI355X.

Workload: inverse homotopy flow dX/dt = X (I - A) X, X(0) = I, T = 1, on the
n = 4096 SPD matrix with lam ~ U[0.05, 4] (seed 2); N = 64 slices, one
forward-Euler coarse step and 16 RK4 fine steps per slice; all slice fine
solves of an iteration batched in one grouped GEMM launch per product, the
launches of one RK4 step replayed from a hipGraph; FP64 correction; the
solve stops when max_n ||U^{k+1}_n - U^k_n||_F / ||U^{k+1}_n||_F <= 1e-8.
Products run in FP64 on MFMA by default: with FP32 products parareal
converges to the FP32 fine solution, 1.8e-6 away from the FP64 one, so only
the FP64 run reaches 1e-8 relative error (--dtype selects another).

One step = one parareal iteration (the batched fine phase over the live
slices, the FP64 correction sweep, the stop test).  The timed region holds
whole converged solves run back to back, about 9 iterations each: solves
are added until `--steps` iterations are covered, unless the next solve
would end past the wall-clock budget (--budget-s, counted from the start of
the process, leaving room for the CPU baseline); `steps` reports the
iterations actually timed.  Warm-up: min(--warmup, 2) iterations of a
truncated solve (workspace allocation, autotuning, graph instantiation).

value = converged solves / timed wall time.  roofline: the fine-step GEMM
launches (affine and RK4-epilogue products of every RK4 step), timed with
HIP events on the solve's stream around each hipGraph replay of one RK4
step; achieved = algorithmic flops (2 n^3 per slice product) / time.

learned_vs_euler (default workload only, after the timed region and the
CPU baseline, if it ends within --learned-budget-s of the process start):
the learned coarse step against forward Euler on the n = 2048 homotopy
(N = 128 slices, 8 RK4 steps per slice, FP64, to increment 1e-8), each
solve timed after one warm-up solve of the flow, with the iteration counts,
the wall times and each result's distance from the serial fine solution.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

T_PROCESS = time.time()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# TFLOP/s, dense MFMA; split BF16 does three BF16 products per algorithmic one
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.0, "f16": 2516.0, "bf16x3": 2516.0 / 3}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
METRIC = "parareal solves/s + MFMA TFLOP/s at 1e-8 rel err; learned vs Euler coarse"


def log(msg):
    print("[bench %6.1fs] %s" % (time.time() - T_PROCESS, msg), file=sys.stderr, flush=True)


def traffic_for(kernel_key, items_per_launch):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE counters
    recorded in profiles/traffic.json (bytes per slice product, calibrated
    against a copy kernel of known size), scaled to this run's products per
    launch; None when the GEMM source changed since the counters were taken."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent:
        return None
    src = open(os.path.join(ROOT, "paper_1505_07959_amd", "csrc", "gemm.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != ent.get("gemm_sha256"):
        return None
    return ent["bytes_per_item"] * items_per_launch


def cpu_baseline(A, n, fine_steps_total, coarse_steps_total, sample_steps):
    """Time the oracle's matrix RK4 step (numpy FP64) on a bounded sample and
    scale to one solve of the same discrete method."""
    import numpy as np
    from oracle import MatrixAlgebra, HOMOTOPY, integrators
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    alg = MatrixAlgebra(n)
    X = np.eye(n)
    h = 1.0 / 1024
    M = A - np.eye(n)
    t0 = time.perf_counter()
    for _ in range(sample_steps):
        X = integrators.rk4_step(alg, HOMOTOPY, X, A, h, M)
    t_step = (time.perf_counter() - t0) / sample_steps
    # one Euler step = 2 of the 8 products of an RK4 step
    t_solve = t_step * (fine_steps_total + 0.25 * coarse_steps_total)
    # the same on one core: one of the eight products of an RK4 step, timed
    # with the BLAS limited to one thread and scaled by 8
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            alg.mul(X, M)
            t_prod = time.perf_counter() - t1
        one = 1.0 / (8.0 * t_prod * (fine_steps_total + 0.25 * coarse_steps_total))
    except Exception:
        pass
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "value_one_core": one,
            "sample": "%d RK4 steps of the n=%d matrix oracle (numpy FP64, %.2f s/step), scaled by the %d RK4 "
                      "and %d Euler steps of one GPU solve; one core: one product of an RK4 step at one BLAS "
                      "thread, scaled by 8" % (sample_steps, n, t_step, fine_steps_total, coarse_steps_total)}


def plan_next_solve(now, solve_s, steps_done, steps_target, budget_s, reserve_s):
    """Whether another whole solve goes into the timed region: more steps are
    wanted and, at the last solve's duration, it ends within the budget
    (seconds since process start) with `reserve_s` left over."""
    if steps_done >= steps_target:
        return False
    return now + solve_s + reserve_s <= budget_s


LEARNED_LEG_S = 75.0  # the learned-vs-Euler leg's wall time, with margin (about 55 s measured)


def plan_learned_leg(now, budget_s, est_s=LEARNED_LEG_S):
    """Whether the learned-vs-Euler leg, started `now` seconds after the
    process start, is expected to end within `budget_s`."""
    return now + est_s <= budget_s


def learned_leg(fm):
    """The learned coarse step against forward Euler on the n = 2048 homotopy
    (N = 128, S = 8, FP64, to 1e-8), each solve after a warm-up solve."""
    from paper_1505_07959_amd import measure_rows
    rows = measure_rows.learned_vs_euler(fm.FM_FLOW_INV_HOMOTOPY)
    by = {("learned" if r["workload"].endswith("_learned") else "euler"): r for r in rows}
    learned = {"workload": "inverse homotopy n=2048 SPD lam~loguniform[1e-2,10] seed 4, N=128 slices, RK4 8 "
                           "steps/slice, FP64 products, stop at increment <= 1e-08; network "
                           "models/homotopy_n256.fmw (trained at n=256)",
               "serial_fine_seconds": by["euler"]["serial_fine_seconds"]}
    for k in ("euler", "learned"):
        r = by[k]
        learned[k] = {"iterations": r["iterations"], "seconds": r["seconds"], "status": r["status"],
                      "restarts": r["restarts"], "rel_diff_vs_serial_fine": r["rel_diff_vs_serial_fine"]}
    learned["learned_fewer_iterations_and_faster"] = (
        learned["learned"]["iterations"] < learned["euler"]["iterations"]
        and learned["learned"]["seconds"] < learned["euler"]["seconds"])
    log("learned %d iterations %.1f s, Euler %d iterations %.1f s" %
        (learned["learned"]["iterations"], learned["learned"]["seconds"],
         learned["euler"]["iterations"], learned["euler"]["seconds"]))
    return learned


def solve_work(n, N, S, iters):
    """Fine RK4 steps and coarse Euler steps of a solve of `iters` iterations:
    iteration k re-solves the slices n >= k; the sweep of iteration k takes a
    coarse step on every slice after the k-th, Step 0 on all N."""
    fine = sum(N - k for k in range(iters)) * S
    coarse = N + sum(N - k - 1 for k in range(iters))
    return fine, coarse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9, help="parareal iterations to time (whole solves)")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up iterations (at most 2 are run)")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget from process start: no timed solve is started that would end later")
    ap.add_argument("--dtype", default="f64", choices=["f32", "f64", "bf16", "f16", "bf16x3"])
    ap.add_argument("--coarse", default="euler", choices=["euler", "learned"])
    ap.add_argument("--tile", default=None, help="fixed product tile <bm>x<bk> instead of the autotuned one")
    ap.add_argument("--coarse-f64", action="store_true", help="coarse-step products in FP64 (FP32/16-bit runs)")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--fine-steps", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=64)
    ap.add_argument("--cpu-sample-steps", type=int, default=12,
                    help="oracle RK4 steps timed for the CPU baseline (about 10-13 s of CPU work at n=4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-Euler leg")
    ap.add_argument("--learned-budget-s", type=float, default=540.0,
                    help="wall-clock limit from process start for the learned-vs-Euler leg")
    ap.add_argument("--serial", action="store_true",
                    help="also time the serial fine solve after the benchmark (off by default: its one-product "
                         "launches of the same kernel would blend into a profile's per-kernel average)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (time slices would shard over "
              "GPUs, one range of slices per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1505_07959_amd import fm, inputs

    n, N, S = args.n, args.slices, args.fine_steps
    log("building input n=%d" % n)
    A, Q, lam = inputs.large_problem(n) if n == 4096 else inputs.spd(n, "uniform", 0.05, 4.0, 2)
    Ad = torch.from_numpy(A).cuda()
    out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    coarse = fm.FM_COARSE_LEARNED if args.coarse == "learned" else fm.FM_COARSE_EULER
    prm = {"T": 1.0, "N": N, "coarse_steps": 1, "fine_steps": S, "max_iter": args.max_iter, "tol": args.tol,
           "coarse": coarse, "max_refine": 0}
    opts = "timing=1;verbose=1" + (";tile=" + args.tile if args.tile else "") + \
           (";coarse_f64=1" if args.coarse_f64 else "")
    if coarse == fm.FM_COARSE_LEARNED:
        opts += ";coarse_model=" + os.path.join(ROOT, "paper_1505_07959_amd", "models", "homotopy_n256.fmw")
    log("creating the flow (autotuning the product tiles)")
    h = fm.fm_flow_create([(fm.FM_FLOW_INV_HOMOTOPY, Ad)], args.dtype, opts)
    stream = torch.cuda.current_stream()

    def one(max_iter):
        st, stats = fm.fm_parareal_solve(h, None, [out], [dict(prm, max_iter=max_iter)], stream=stream)
        return st, stats[0]

    warm = min(args.warmup, 2)
    if warm > 0:
        t = time.perf_counter()
        st, s = one(warm)
        log("warm-up: %d iterations in %.2f s (status %d)" % (s["iters"], time.perf_counter() - t, st))

    # timed region: whole solves, back to back
    reserve = 0.0 if args.no_cpu_baseline else 30.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solves = []
    last = None
    while True:
        ts = time.perf_counter()
        st, s = one(args.max_iter)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        solves.append((st, s, dt))
        last = dt
        done = sum(x[1]["iters"] for x in solves)
        log("solve %d: %d iterations, increment %.3e, status %d, %.2f s (%d steps timed)" %
            (len(solves), s["iters"], s["increment"], st, dt, done))
        if not plan_next_solve(time.time() - T_PROCESS, last, done, args.steps, args.budget_s, reserve):
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps = sum(x[1]["iters"] for x in solves)
    if steps < args.steps:
        log("wall-clock budget: %d of %d requested steps timed (%d whole solves)" % (steps, args.steps, len(solves)))

    # outside the timed region: the serial fine solve that the parareal
    # iteration converges to (N*S RK4 steps from X0 = I on one GPU), for the
    # comparison a single GPU can show; parareal pays off when slices run on
    # separate GPUs
    serial = None
    if args.serial:
        log("serial fine solve: %d RK4 steps" % (N * S))
        X0 = torch.eye(n, dtype=torch.float64, device="cuda")
        Xs = torch.empty_like(X0)
        fm.fm_fine_propagate(h, 1.0 / (N * S), 0.0, 1, [X0], [Xs], stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fm.fm_fine_propagate(h, 1.0, 0.0, N * S, [X0], [Xs], stream=stream)
        torch.cuda.synchronize()
        tser = time.perf_counter() - t
        serial = {"seconds": tser, "rk4_steps": N * S, "tflops": N * S * 16.0 * n ** 3 / tser / 1e12,
                  "rel_diff_vs_parareal": float(torch.linalg.norm(out - Xs) / torch.linalg.norm(Xs))}
        log("serial fine: %.2f s, rel diff %.2e" % (tser, serial["rel_diff_vs_parareal"]))
    fm.fm_destroy(h)

    converged = [x for x in solves if x[0] == fm.FM_OK]
    solves_per_s = len(converged) / elapsed
    launches = sum(x[1]["fine_launches"] for x in solves)
    fine_ms = sum(x[1]["fine_ms"] for x in solves)
    fine_flops = sum(x[1]["fine_flops"] for x in solves)
    avg_launch_ms = fine_ms / max(1, launches)
    flops_per_launch = fine_flops / max(1, launches)
    achieved = fine_flops / (fine_ms * 1e-3) / 1e12 if fine_ms > 0 else 0.0
    iters = [x[1]["iters"] for x in solves]
    s = solves[-1][1]
    fine_steps_total, coarse_steps_total = solve_work(n, N, S, s["iters"])
    total_fine_flops = sum(solve_work(n, N, S, k)[0] for k in iters) * 16.0 * n ** 3
    log("iterations per solve %s, hist %s" % (iters, ["%.1e" % x for x in s["hist"]]))
    log("fine-step GEMM: %d launches, avg %.3f ms, %.1f TFLOP/s; fine phases %.1f s of %.1f s timed" %
        (launches, avg_launch_ms, achieved, sum(x[1]["fine_phase_ms"] for x in solves) / 1e3, elapsed))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (%d oracle RK4 steps at n=%d)" % (args.cpu_sample_steps, n))
        cpu = cpu_baseline(A, n, fine_steps_total, coarse_steps_total, args.cpu_sample_steps)

    # outside the timed region: learned vs Euler coarse step (the default
    # workload only, so that runs of other shapes keep their launches alone)
    learned = None
    default_run = (args.dtype, n, N, S, args.coarse, args.tol, args.max_iter, args.tile, args.coarse_f64) == \
        ("f64", 4096, 64, 16, "euler", 1e-8, 64, None, False)
    if default_run and not args.no_learned:
        now = time.time() - T_PROCESS
        if plan_learned_leg(now, args.learned_budget_s):
            log("learned vs Euler coarse step: n=2048 homotopy, N=128, S=8, FP64, to 1e-8")
            try:
                learned = learned_leg(fm)
            except Exception as e:  # the extra leg never costs the benchmark line
                log("learned-vs-Euler leg failed: %r" % (e,))
                learned = {"error": repr(e)}
        else:
            log("learned-vs-Euler leg skipped: it would end past %.0f s" % args.learned_budget_s)

    key = "gemm_%s_fine_step_n%d" % (args.dtype, n)
    res = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "inverse homotopy dX/dt=X(I-A)X, n=%d SPD lam~U[0.05,4] seed 2, N=%d slices, "
                               "RK4 %d steps/slice, %s coarse 1 step/slice, %s MFMA products, %s, FP64 correction, "
                               "stop at increment <= %g" % (n, N, S, args.coarse, args.dtype,
                                                            "FP32 fine-solve state" if args.dtype in ("bf16", "f16", "bf16x3")
                                                            else "FP64 state", args.tol),
                   "step": "one parareal iteration (batched fine phase, FP64 correction sweep, stop test); "
                           "whole converged solves timed back to back",
                   "n": n, "slices": N, "fine_steps": S, "coarse_steps": 1, "coarse": args.coarse, "tol": args.tol,
                   "solves_timed": len(solves), "solves_converged": len(converged),
                   "iterations_per_solve": iters, "seconds_per_solve": [round(x[2], 3) for x in solves],
                   "steps_requested": args.steps, "warmup_requested": args.warmup,
                   "learned_restarts": [x[1]["learned_restarts"] for x in solves],
                   "fine_tflops_whole_solve": total_fine_flops / elapsed / 1e12},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.dtype], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[args.dtype],
                     "traffic": traffic_for(key, flops_per_launch / (2.0 * n ** 3)),
                     "kernel": "gemm_kernel fine-step launches (affine + RK4-epilogue products), HIP events around "
                               "each graph replay of one RK4 step: %d launches, avg %.3f ms, %.3e flop/launch"
                               % (launches, avg_launch_ms, flops_per_launch)},
        "cpu_baseline": cpu,
        "serial_fine": serial,
        "learned_vs_euler": learned,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
