"""Benchmark of the mobility solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload random64]

A step is one full mobility solve (incident density, right-hand side, GMRES to
the relative residual tolerance, velocities) with the loads already resident in
HBM; setup (singular operators, block inverses) happens once before timing.
Prints ONE JSON line.  ``value`` is the whole-solve pair-interaction throughput of
the plain float64 solve (off-body pair interactions evaluated by all of its sums,
divided by its wall time).  The same run also times the mixed-precision
(GMRES-IR) solve at the same tolerance, the roofline of the dominant kernel (the
float64 traction sum, timed with HIP events on the library stream), and the FP64
NumPy oracle's pair rate on the host (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mobility solve time @1e-8 rel. residual (mixed+learned vs FP64); Gpairs/s"
FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32 (packed issue)
TRACTION_FLOPS_PER_PAIR = 30


def _cpu_baseline(w, budget_s):
    """Oracle traction sum (float64 NumPy) on a bounded sample of targets of the
    same workload; returns Gpairs/s on the host."""
    from oracle import farfield as ff
    from tests.helpers import oracle_problem  # geometry only, no singular operators
    prob = oracle_problem(w, with_ops=False)
    rng = np.random.default_rng(0)
    mu = rng.standard_normal((prob.N, 3))
    q = prob.w[:, None] * mu
    order = rng.permutation(prob.N)
    done, pairs = 0, 0.0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < prob.N:
        idx = order[done:done + 64]
        ff.traction_sum(prob.X[idx], prob.Nn[idx], prob.X, q, prob.body[idx], prob.body)
        pairs += len(idx) * (prob.N - prob.M)
        done += len(idx)
    dt = time.perf_counter() - t0
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle float64 traction sum at {done} of {prob.N} targets against all "
                      f"{prob.N} sources ({pairs:.3e} pairs, {dt:.1f} s, NumPy single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="random64")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1606_07428_amd import inputs, rbm

    w = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] workload {args.workload}: n={len(w['shape_id'])} p={w['p']}", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    s64 = rbm.solver_for(w, tol=args.tol, precision=rbm.FP64, guess=rbm.GUESS_BLOCKDIAG)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    FT = torch.as_tensor(np.asarray(w["FT"], dtype=np.float64), device=dev)
    VW = torch.zeros_like(FT)

    def run(solver, steps, out):
        infos = []
        for _ in range(steps):
            infos.append(solver.solve_dev(FT, out))
        return infos

    run(s64, args.warmup, VW)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = run(s64, args.steps, VW)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    VW64 = VW.cpu().numpy().copy()
    print(f"[bench] fp64: {dt / args.steps * 1e3:.3f} ms/solve, iters {infos[-1]['iters']}",
          file=sys.stderr, flush=True)

    pairs = sum(i["far_pairs"] for i in infos)
    ms_trac = sum(i["ms_traction"] for i in infos)
    n_trac = sum(i["n_traction"] for i in infos)
    ppl = infos[-1]["pairs_per_launch"]
    trac_avg_s = ms_trac / max(n_trac, 1) / 1e3
    achieved = TRACTION_FLOPS_PER_PAIR * ppl / trac_avg_s / 1e12
    result = {
        "metric": METRIC,
        "value": pairs / dt / 1e9,
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "bodies": int(len(w["shape_id"])), "p": w["p"],
                   "points": int(len(w["shape_id"]) * 2 * w["p"] * (w["p"] + 1)),
                   "tol": args.tol, "precision": "fp64", "guess": "block-diagonal"},
        "roofline": {"bound": "alu", "kernel": "k_far<double, traction>",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "launch_ms": trac_avg_s * 1e3, "pairs_per_launch": ppl,
                     "flops_per_pair": TRACTION_FLOPS_PER_PAIR},
        "solve": {"fp64_ms": dt / args.steps * 1e3, "iters": infos[-1]["iters"],
                  "matvecs": infos[-1]["matvecs"], "rel_residual": infos[-1]["rel_residual"],
                  "solves_per_s": args.steps / dt,
                  "matvecs_per_s": sum(i["matvecs"] for i in infos) / dt,
                  "traction_gpairs_per_s": ppl / trac_avg_s / 1e9,
                  "setup_s": setup_s},
    }
    s64.close()
    del s64
    torch.cuda.empty_cache()

    if not args.no_mixed:
        s32 = rbm.solver_for(w, tol=args.tol, precision=rbm.MIXED_FP32, guess=rbm.GUESS_BLOCKDIAG)
        run(s32, args.warmup, VW)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf32 = run(s32, args.steps, VW)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t0
        VW32 = VW.cpu().numpy()
        err = float(np.abs(VW32 - VW64).max() / np.abs(VW64).max())
        ms32 = sum(i["ms_traction"] for i in inf32)
        n32 = sum(i["n_traction"] for i in inf32)
        result["solve"].update({
            "mixed_fp32_ms": dt32 / args.steps * 1e3, "mixed_iters": inf32[-1]["iters"],
            "mixed_refinements": inf32[-1]["refinements"],
            "mixed_rel_residual": inf32[-1]["rel_residual"],
            "mixed_vs_fp64_velocity_rel_err": err,
            "mixed_speedup": (dt / args.steps) / (dt32 / args.steps),
        })
        # the fp32 launches include the fp64 residual launches; report the mixed average
        result["solve"]["mixed_traction_launch_ms_avg"] = ms32 / max(n32, 1)
        s32.close()
        print(f"[bench] mixed fp32: {dt32 / args.steps * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)

    if not args.no_cpu:
        result["cpu_baseline"] = _cpu_baseline(w, args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
