"""Timing of the paper's own examples and the linear-flow algorithms on one
GPU (one JSON line per workload).  Inputs are the seeded synthetic matrices
of ``inputs``; times are wall-clock around the blocking library calls with
the inputs resident on the device.

    python -m paper_1505_07959_amd.measure_rows [--only NAME ...]
"""

import argparse
import json
import time

import numpy as np
import torch

from paper_1505_07959_amd import fm, inputs


def _timed(fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def _serial_fine(flow, ns, T, steps):
    """GPU wall time of the serial fine solve the parareal iteration converges
    to: all N*S RK4 steps from X0 = I over [0, T] for every problem of the
    flow, in one fm_fine_propagate call (after a one-step warm-up)."""
    X0 = [torch.eye(n, dtype=torch.float64, device="cuda") for n in ns]
    Xs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in ns]
    fm.fm_fine_propagate(flow, T / steps, 0.0, 1, X0, Xs)
    _, sec = _timed(lambda: fm.fm_fine_propagate(flow, T, 0.0, steps, X0, Xs))
    return sec, Xs


def _solve(kind, A, prm, dtype="f64", options="timing=1"):
    n = A.shape[0]
    h = fm.fm_flow_create([(kind, A)], dtype, options)
    try:
        out = torch.empty((n, n), dtype=torch.float64, device="cuda")
        fm.fm_parareal_solve(h, None, [out], [dict(prm, tol=0.0, max_iter=1)])   # warm-up (autotune, graphs)
        (st, stats), sec = _timed(lambda: fm.fm_parareal_solve(h, None, [out], [prm]))
        return stats[0], sec
    finally:
        fm.fm_destroy(h)


def example1():
    """Sec. 2, Example 1 at the paper's sizes: n = 80, N = 25, J = 200, Euler."""
    A = torch.from_numpy(inputs.laplacian_1d(80) / 2 ** 10).cuda()
    s, sec = _solve(fm.FM_FLOW_INV_HOMOTOPY, A, {"T": 1.0, "N": 25, "fine_steps": 200, "max_iter": 25,
                                                 "tol": 1e-10, "fine_method": fm.FM_FINE_EULER})
    return {"workload": "example1_laplacian80_euler_N25_J200", "iterations": s["iters"], "seconds": sec,
            "note": "latency-bound: 5000 Euler steps of 80 x 80 products per fine sweep"}


def example2_cn():
    """Sec. 2, Example 2 at the paper's sizes: exp(B), B = -A / 2^10 with the
    Example 1 Laplacian (n = 80), N = 25, J = 200, Crank-Nicolson fine and
    coarse steps, to increment 1e-10."""
    B = torch.from_numpy(-inputs.laplacian_1d(80) / 2 ** 10).cuda()
    s, sec = _solve(fm.FM_FLOW_EXP, B, {"T": 1.0, "N": 25, "fine_steps": 200, "max_iter": 25, "tol": 1e-10,
                                        "fine_method": fm.FM_FINE_CN, "coarse": fm.FM_COARSE_CN})
    return {"workload": "example2_laplacian80_crank_nicolson_N25_J200", "iterations": s["iters"], "seconds": sec,
            "note": "latency-bound: 5000 Crank-Nicolson steps of 80 x 80 products per fine sweep"}


def exp_variants(n=2048):
    """exp(T A) by the exponential flow, A = -(SPD, lam in [0.05, 4]), N = 16,
    16 RK4 steps per slice, FP64, to increment 1e-10: classical vs modified."""
    A0, Q, lam = inputs.spd(n, "uniform", 0.05, 4.0, 81)
    A = torch.from_numpy(-A0).cuda()
    out = []
    for variant, name in ((fm.FM_PARAREAL_CLASSICAL, "classical"), (fm.FM_PARAREAL_MODIFIED, "modified")):
        s, sec = _solve(fm.FM_FLOW_EXP, A, {"T": 1.0, "N": 16, "fine_steps": 16, "max_iter": 16, "tol": 1e-10,
                                            "variant": variant})
        tf = s["fine_flops"] / (s["fine_ms"] * 1e-3) / 1e12 if s["fine_ms"] > 0 else None
        out.append({"workload": "exp_flow_n%d_N16_S16_f64_%s" % (n, name), "iterations": s["iters"],
                    "basis": s["basis_size"], "seconds": sec, "fine_gemm_tflops": tf})
    return out


def aima(m=63, steps=200):
    """Alg. 8 on the 5-point Laplacian of an m x m grid scaled by its
    Frobenius norm, dt = 0.1, exact initial error switched off at t = 1:
    two products per step for the first 10 steps, one after."""
    L = inputs.laplacian_2d(m)
    A = L / np.linalg.norm(L)
    n = A.shape[0]
    E = torch.from_numpy(np.linalg.inv(A)).cuda()
    Ad = torch.from_numpy(A).cuda()
    res = []
    for dtype in ("f64", "f32"):
        h = fm.fm_flow_create([(fm.FM_FLOW_INV_LINEAR, Ad)], dtype)
        try:
            X = torch.empty((n, n), dtype=torch.float64, device="cuda")
            fm.fm_aima(h, None, [E], 0.1, 2, [X])
            _, sec = _timed(lambda: fm.fm_aima(h, None, [E], 0.1, steps, [X], accel_steps=10))
        finally:
            fm.fm_destroy(h)
        acc = min(steps, 10)   # two products per step while the accelerator is on, one after
        fl = (2 * acc + (steps - acc)) * 2.0 * n ** 3
        res.append({"workload": "aima_laplacian2d_n%d_%s" % (n, dtype), "steps": steps, "seconds": sec,
                    "ms_per_step": 1e3 * sec / steps, "tflops": fl / sec / 1e12})
    return res


def cosine(n=2048):
    """Alg. 5: cos(A), A symmetric with ||A||_inf ~ 8 (m = 3), N = 10, 100
    RK4 steps per slice on the 2n x 2n system, FP64, tol 1e-12."""
    A0, Q, lam = inputs.spd(n, "uniform", -4.0, 4.0, 82)
    A = torch.from_numpy(A0).cuda()
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    out = []
    for variant, name in ((fm.FM_PARAREAL_CLASSICAL, "classical"), (fm.FM_PARAREAL_MODIFIED, "modified")):
        prm = {"N": 10, "fine_steps": 100, "max_iter": 10, "tol": 1e-12, "variant": variant}
        fm.fm_cos(A, C, dict(prm, max_iter=1, tol=0.0))
        (st, m, s), sec = _timed(lambda: fm.fm_cos(A, C, prm))
        ref = (Q * np.cos(lam)) @ Q.T
        err = float(np.abs(C.cpu().numpy() - ref).max() / np.abs(ref).max())
        out.append({"workload": "cos_n%d_N10_J100_f64_%s" % (n, name), "m": m, "iterations": s["iters"],
                    "basis": s["basis_size"], "seconds": sec, "max_rel_error": err})
    return out


def batched(count=512, tol=1e-3):
    """The batched workload: 512 problems, n uniform on {32, ..., 512}, half
    inverse homotopy (T = 1), half A - X^2 (T = 20), BF16 products, N = 64,
    8 RK4 steps per slice, to increment 1e-3, then FP64 refinement."""
    cases = [inputs.batched_instance(i) for i in range(count)]
    prm = [{"T": T, "N": 64, "fine_steps": 8, "coarse_steps": 1 if k == fm.FM_FLOW_INV_HOMOTOPY else 2,
            "max_iter": 64, "tol": tol, "max_refine": 6, "refine_tol": 1e-13} for k, T, *_ in cases]
    flow = fm.fm_flow_create([(k, torch.from_numpy(A).cuda()) for k, T, A, Q, lam in cases], "bf16")
    try:
        outs = [torch.empty((c[2].shape[0],) * 2, dtype=torch.float64, device="cuda") for c in cases]
        fm.fm_parareal_solve(flow, None, outs, [dict(p, max_iter=1, max_refine=0) for p in prm])
        (st, stats), sec = _timed(lambda: fm.fm_parareal_solve(flow, None, outs, prm))
    finally:
        fm.fm_destroy(flow)
    # serial fine solves of the same problems (one flow per kind: the two
    # halves end at different T)
    serial = 0.0
    for kind, T in ((fm.FM_FLOW_INV_HOMOTOPY, 1.0), (fm.FM_FLOW_SQRT_STEADY, 20.0)):
        sub = [c for c in cases if c[0] == kind]
        f2 = fm.fm_flow_create([(kind, torch.from_numpy(A).cuda()) for k, T2, A, Q, lam in sub], "bf16")
        try:
            serial += _serial_fine(f2, [c[2].shape[0] for c in sub], T, 64 * 8)[0]
        finally:
            fm.fm_destroy(f2)
    its = [s["iters"] for s in stats]
    return {"workload": "batched%d_bf16_N64_S8_tol%g_refined" % (count, tol), "seconds": sec,
            "serial_fine_seconds": serial, "solves_per_s": count / sec,
            "iterations_max": max(its), "iterations_mean": float(np.mean(its)),
            "refine_steps_max": max(s["refine_steps"] for s in stats),
            "residual_max": max(s["residual"] for s in stats)}


def learned_vs_euler(kind=fm.FM_FLOW_INV_HOMOTOPY, dtype=None, tol=None, options=""):
    """Learned vs Euler coarse step: the n = 2048 homotopy (N = 128, S = 8,
    FP64, to 1e-8) or the n = 8192 X - XAX flow (N = 32, S = 16, T = 30,
    FP16 products, to 1e-3), each after one warm-up solve of the flow."""
    from paper_1505_07959_amd import eval_coarse
    if kind == fm.FM_FLOW_INV_HOMOTOPY:
        n, N, S, T, dt, tl = 2048, 128, 8, 1.0, "f64", 1e-8
        A = inputs.learned_eval_problem(n)[0]
    else:
        n, N, S, T, dt, tl = 8192, 32, 16, 30.0, "f16", 1e-3
        A = inputs.steady_problem(n)[0]
    dt = dtype or dt
    tol = tol or tl
    Ad = torch.from_numpy(A).cuda()
    model = eval_coarse.DEFAULT_MODEL[kind]
    flow = fm.fm_flow_create([(kind, Ad)], dt, "coarse_model=%s" % model + (";" + options if options else ""))
    out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    res = []
    try:
        fm.fm_parareal_solve(flow, None, [out], [{"T": T, "N": N, "fine_steps": S, "max_iter": 1, "tol": 0.0}])
        serial, Xs = _serial_fine(flow, [n], T, N * S)
        for name, coarse in (("euler", fm.FM_COARSE_EULER), ("learned", fm.FM_COARSE_LEARNED)):
            prm = {"T": T, "N": N, "fine_steps": S, "max_iter": N, "tol": tol, "coarse": coarse}
            (st, stats), sec = _timed(lambda: fm.fm_parareal_solve(flow, None, [out], [prm]))
            s = stats[0]
            res.append({"workload": "%s_n%d_N%d_S%d_%s_tol%g_%s%s" % ("homotopy" if kind == 1 else "steady", n, N, S,
                                                                      dt, tol, name, "_" + options if options else ""),
                        "iterations": s["iters"], "seconds": sec, "serial_fine_seconds": serial,
                        "rel_diff_vs_serial_fine": float(torch.linalg.norm(out - Xs[0]) / torch.linalg.norm(Xs[0])),
                        "restarts": s["learned_restarts"], "status": st})
    finally:
        fm.fm_destroy(flow)
    return res


def vendor_gemm():
    """Reference for the products: torch.matmul (the vendor BLAS) on seeded
    random n x n products -- FP16 and BF16 at n = 4096 (16 per call), FP16 at
    n = 8192 (4 per call), FP64 at n = 4096 (4 per call) -- and, for the
    RK4-epilogue product, the same FP16 products followed by the stage
    update as separate elementwise operations (k = -P, accumulator += 2 k,
    next operand = x + h/2 k in FP16, FP32 state), the unfused equivalent of
    one stage-2 launch.  The rate random data sustains on this chip (its
    clock drops under the matrix units' load) bounds what the fine-step
    products can reach."""
    out = []

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for name, dt, n, batch in (("f16", torch.float16, 4096, 16), ("bf16", torch.bfloat16, 4096, 16),
                               ("f16", torch.float16, 8192, 4), ("f64", torch.float64, 4096, 4)):
        g = torch.Generator(device="cuda").manual_seed(7)
        a = torch.randn(batch, n, n, device="cuda", dtype=torch.float32, generator=g).to(dt)
        b = torch.randn(batch, n, n, device="cuda", dtype=torch.float32, generator=g).to(dt)
        c = torch.empty_like(a)
        ms = timed(lambda: torch.matmul(a, b, out=c))
        out.append({"workload": "torch_matmul_%s_%dx%d" % (name, batch, n), "ms_per_call": ms,
                    "tflops": 2.0 * batch * n ** 3 / (ms * 1e-3) / 1e12})
        if name == "f16" and n == 4096:
            x = torch.randn(batch, n, n, device="cuda", dtype=torch.float32, generator=g)
            kq = torch.randn(batch, n, n, device="cuda", dtype=torch.float32, generator=g)
            y = torch.empty_like(a)
            h = 1e-3

            def stage():
                torch.matmul(a, b, out=c)
                k = -c.float()
                kq.add_(k, alpha=2.0)
                torch.add(x, k, alpha=0.5 * h, out=k)
                y.copy_(k)

            ms = timed(stage)
            out.append({"workload": "torch_matmul_f16_%dx%d_then_rk4_stage_update" % (batch, n), "ms_per_call": ms,
                        "tflops": 2.0 * batch * n ** 3 / (ms * 1e-3) / 1e12})
            del x, kq, y
        del a, b, c
        torch.cuda.empty_cache()
    return out


ROWS = {"example1": example1, "example2_cn": example2_cn, "exp": exp_variants, "aima": aima, "cos": cosine, "batched": batched,
        "batched_tol1e-2": lambda: batched(tol=1e-2),
        "learned": lambda: learned_vs_euler(fm.FM_FLOW_INV_HOMOTOPY),
        "learned_f32": lambda: learned_vs_euler(fm.FM_FLOW_INV_HOMOTOPY, "f32", 1e-6),
        "learned_f32_coarse64": lambda: learned_vs_euler(fm.FM_FLOW_INV_HOMOTOPY, "f32", 1e-7, "coarse_f64=1"),
        "learned_steady": lambda: learned_vs_euler(fm.FM_FLOW_INV_STEADY),
        "learned_steady_coarse64": lambda: learned_vs_euler(fm.FM_FLOW_INV_STEADY, options="coarse_f64=1"),
        "vendor_gemm": vendor_gemm}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=list(ROWS))
    a = ap.parse_args()
    for name in a.only:
        r = ROWS[name]()
        for line in (r if isinstance(r, list) else [r]):
            print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
