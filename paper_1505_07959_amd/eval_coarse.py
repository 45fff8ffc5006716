"""Learned versus Euler coarse propagator in parareal on one MI355X.

Runs fm_parareal_solve twice on the same problem (inverse homotopy,
n = 2048 SPD with lam ~ loguniform[1e-2, 10], seed 4; N = 128 slices, one
coarse step and 8 RK4 steps per slice) with the Euler and the learned coarse
step, and reports iterations and wall time until the increment
max_n ||U^{k+1}_n - U^k_n||_F / ||U^{k+1}_n||_F falls to `tol`.

Usage: python -m paper_1505_07959_amd.eval_coarse --model models/homotopy_n256.fmw
"""

import argparse
import json
import os
import sys
import time

import torch

from paper_1505_07959_amd import fm, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = {fm.FM_FLOW_INV_HOMOTOPY: os.path.join(HERE, "models", "homotopy_n256.fmw"),
                 fm.FM_FLOW_INV_STEADY: os.path.join(HERE, "models", "steady_n256.fmw")}


def evaluate(model=None, kind=fm.FM_FLOW_INV_HOMOTOPY, n=2048, N=128, S=8, T=1.0, dtype="f64", tol=1e-8,
             max_iter=None, A=None, log=None):
    model = model or DEFAULT_MODEL[kind]
    if A is None:
        A = inputs.learned_eval_problem(n)[0] if kind == fm.FM_FLOW_INV_HOMOTOPY else inputs.steady_problem(n)[0]
    n = A.shape[0]
    Ad = torch.from_numpy(A).cuda()
    out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    flow = fm.fm_flow_create([(kind, Ad)], dtype, "coarse_model=%s;verbose=%d" % (model, 1 if log else 0))
    res = {"n": n, "slices": N, "fine_steps": S, "T": T, "dtype": dtype, "tol": tol, "model": os.path.basename(model)}
    try:
        for name, coarse in (("euler", fm.FM_COARSE_EULER), ("learned", fm.FM_COARSE_LEARNED)):
            prm = {"T": T, "N": N, "fine_steps": S, "coarse_steps": 1, "max_iter": max_iter or N, "tol": tol,
                   "coarse": coarse}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, stats = fm.fm_parareal_solve(flow, None, [out], [prm])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s = stats[0]
            res[name] = {"iterations": s["iters"], "seconds": dt, "status": st, "increments": s["hist"],
                         "learned_slices_last_iteration": s["learned_slices"], "restarts": s["learned_restarts"]}
            if log:
                log("%s coarse: %d iterations, %.2f s, status %d" % (name, s["iters"], dt, st))
    finally:
        fm.fm_destroy(flow)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--model", default=None)
    ap.add_argument("--kind", type=int, default=fm.FM_FLOW_INV_HOMOTOPY)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--slices", type=int, default=128)
    ap.add_argument("--fine-steps", type=int, default=8)
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--tol", type=float, default=1e-8)
    a = ap.parse_args()
    r = evaluate(a.model, a.kind, a.n, a.slices, a.fine_steps, a.T, a.dtype, a.tol,
                 log=lambda m: print("[eval] " + m, file=sys.stderr, flush=True))
    print(json.dumps(r))


if __name__ == "__main__":
    main()
