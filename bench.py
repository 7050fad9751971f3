"""Benchmark of the mobility solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dense4000]
    python bench.py --learned-experiment [--workload sediment512]

A step is one full mobility solve (incident density, right-hand side, GMRES to the
relative residual tolerance 1e-8, velocities) with the loads already resident in
HBM; setup (singular operators, block inverses) happens once before timing.

Default mode (one JSON line), on the 4000-body suspension at 20 % volume fraction with
surfaces 0.1 apart (p = 12, 1.25 M points, near-singular upsampling of order 24 for near
body pairs):
  1. a precision-form context (float32 inner far sums by the fast multipole method of
     order 12, float32 block preconditioner, float64 refinement residuals) runs a short RK4
     trajectory from the configuration, capturing every stage solve, and trains its warm
     start network on them;
  2. at the configuration the trajectory reached (not in the training data) it times K
     solves of the precision form with the learned guess (``ms_per_step``); then, at the
     same state, a stated smaller count of precision-form solves with the block-diagonal
     guess and of plain float64 solves with the block-diagonal guess (float64 direct sums
     throughout);
  3. ``value`` is the off-body pair interactions the float64 solve evaluates divided by the
     learned precision-form solve's time (the float64 solve's work delivered per second);
     ``roofline`` is the far-sum kernel that takes the most time in the timed solves (at
     4000 bodies the fused float64 traction + Stokeslet pass that ends each solve; HIP events
     on the library stream around its launches), ``roofline_others`` the other far-sum
     kernels of the same solves; ``cpu_baseline`` is the FP64 NumPy oracle's traction sum
     on a sample of targets, threaded over the host's cores.
--learned-experiment: paired learned-vs-block-diagonal iteration counts along a
trajectory (train on the first steps, evaluate on the following ones).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mobility solve time @1e-8 rel. residual (mixed+learned vs FP64); Gpairs/s"
FP64_PEAK_TFLOPS = 78.6      # MI355X vector FP64
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32
TRACTION_FLOPS_PER_PAIR = 30
STOKESLET_FLOPS_PER_PAIR = 28
# far-sum kernels of a solve: name, info fields (summed ms, launches), flops per pair, peak,
# the sources their traffic record is tied to
FAR_KERNELS = [
    ("k_far_ts (float64 traction + Stokeslet)", "ms_fused", "n_fused",
     TRACTION_FLOPS_PER_PAIR + STOKESLET_FLOPS_PER_PAIR, FP64_PEAK_TFLOPS,
     ("k_far_fused.hip", "pair.h", "far_plan.h")),
    ("k_far<double, traction>", "ms_traction", "n_traction", TRACTION_FLOPS_PER_PAIR, FP64_PEAK_TFLOPS,
     ("k_far.hip", "pair.h", "far_plan.h")),
    ("k_far<float, traction>", "ms_traction32", "n_traction32", TRACTION_FLOPS_PER_PAIR, FP32_PEAK_TFLOPS,
     ("k_far.hip", "pair.h", "far_plan.h")),
]

# Per workload: near-singular upsampling order (0 = plain smooth rule), fast multipole order
# of the inner far sums (0 = direct float32 sums) and RK4 steps of the training trajectory.
WORKLOAD_DEFAULTS = {
    "dense4000": (24, 12, 2),
    "dense512": (24, 0, 4),
    "ellipsoids1000": (0, 12, 2),
    "sediment512": (0, 0, 4),
    "random64": (0, 0, 8),
}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(w, budget_s, threads):
    """Oracle traction sum (float64 NumPy) on a bounded sample of targets of the same
    workload, the targets split over `threads` host threads; Gpairs/s on the host."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import farfield as ff
    from tests.helpers import oracle_problem  # geometry only, no singular operators
    prob = oracle_problem(w, with_ops=False)
    rng = np.random.default_rng(0)
    mu = rng.standard_normal((prob.N, 3))
    q = prob.w[:, None] * mu
    order = rng.permutation(prob.N)
    chunk = 8

    def work(k):
        done = pairs = 0
        t0 = time.perf_counter()
        pos = k * chunk
        while time.perf_counter() - t0 < budget_s and pos < prob.N:
            idx = order[pos:pos + chunk]
            ff.traction_sum(prob.X[idx], prob.Nn[idx], prob.X, q, prob.body[idx], prob.body)
            pairs += len(idx) * (prob.N - prob.M)
            done += len(idx)
            pos += threads * chunk
        return done, pairs

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(work, range(threads)))
    dt = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    pairs = float(sum(r[1] for r in res))
    return {"value": pairs / dt / 1e9, "unit": "Gpairs/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"oracle float64 traction sum at {done} of {prob.N} targets against all {prob.N} "
                      f"sources ({pairs:.3e} pairs, {dt:.1f} s, NumPy in {threads} threads)"}


def _kernel_source_hash(files=("k_far.hip", "pair.h", "far_plan.h")):
    """sha256 of a far-sum kernel's sources (the kernel file, its pair arithmetic and its
    source-chunk plan)."""
    import hashlib
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(ROOT, "paper_1606_07428_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic(kernel, workload, files):
    """HBM bytes per launch of `kernel` at `workload` from a committed counter summary
    (profiles/traffic_<workload>*.json: FETCH_SIZE and WRITE_SIZE passes, scaled by the
    plain-copy calibration), or None when none exists for the kernel's current sources."""
    import glob
    want = _kernel_source_hash(files)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_{workload}*.json"))):
        try:
            with open(path) as f:
                t = json.load(f)
        except (OSError, ValueError):
            continue
        if t.get("kernel") == kernel and t.get("source_sha256") == want:
            return {"bytes_per_launch": t["fetch_bytes"] + t["write_bytes"], "fetch_bytes": t["fetch_bytes"],
                    "write_bytes": t["write_bytes"], "source": os.path.basename(path)}
    return None


def _rooflines(infl, ppl, workload):
    """Achieved algorithmic FLOP/s of each far-sum kernel over the timed solves (HIP events
    around its launches), largest total time first."""
    out = []
    for name, ms_key, n_key, fpp, peak, files in FAR_KERNELS:
        if name.startswith("k_far<float") and infl[-1]["fmm_applies"]:
            continue  # the inner sums ran as fast multipole evaluations, not this kernel
        ms = sum(i[ms_key] for i in infl)
        n = sum(i[n_key] for i in infl)
        if n == 0:
            continue
        avg_s = ms / n / 1e3
        achieved = fpp * ppl / avg_s / 1e12
        traffic = _traffic(name, workload, files)
        out.append({"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": traffic["bytes_per_launch"] if traffic else None,
                    "traffic_detail": traffic, "launch_ms": avg_s * 1e3, "launches": n,
                    "pairs_per_launch": ppl, "flops_per_pair": fpp, "total_ms": ms})
    out.sort(key=lambda r: -r["total_ms"])
    return out


def _timed(torch, solver, FT, VW, steps, warmup):
    for _ in range(warmup):
        solver.solve_dev(FT, VW)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for k in range(steps):
        infos.append(solver.solve_dev(FT, VW))
        if steps > 4 and solver.N > 200_000:
            _log(f"  solve {k + 1}/{steps}: {infos[-1]['ms_total']:.0f} ms, {infos[-1]['iters']} it")
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos


def _spread(infos):
    """Median and interquartile range (ms) of the per-solve times recorded by the library's
    stream events around each solve (the timed bracket itself is not changed)."""
    t = np.sort(np.array([i["ms_total"] for i in infos]))
    q1, med, q3 = np.percentile(t, [25, 50, 75])
    return float(med), float(q3 - q1)


def _dt_rule(VW):
    """Time step from the first solve: 0.02 / max_i |v_i - mean v|."""
    v = VW[:, :3]
    return 0.02 / max(np.abs(v - v.mean(axis=0)).max(), 1e-12)


def _train_on_trajectory(rbm, torch, w, FT, tol, steps, epochs, lr, precision, p_up=0, near_factor=5.0,
                         fmm_order=0):
    t0 = time.perf_counter()
    s = rbm.solver_for(w, tol=tol, precision=precision, guess=rbm.GUESS_BLOCKDIAG, p_up=p_up,
                       near_factor=near_factor, fmm_order=fmm_order)
    s.learned_bind(k_nbr=8, hidden=256, n_hidden=3, capacity=max(4 * steps * s.n, 1),
                   batch_max=1024, seed=7)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    VW = torch.zeros_like(FT)
    s.solve_dev(FT, VW)
    dt = _dt_rule(VW.cpu().numpy())
    _log(f"training trajectory: setup {setup_s:.1f} s, dt {dt:.4g}, {steps} RK4 steps")
    s.learned_set_capture(True)
    t0 = time.perf_counter()
    for k in range(steps):
        s.step_rk4(dt, FT)
        torch.cuda.synchronize()
        _log(f"  RK4 step {k + 1}/{steps} done ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t_traj = time.perf_counter() - t0
    s.learned_set_capture(False)
    t0 = time.perf_counter()
    loss0 = s.learned_train(1, 256, lr)
    loss = s.learned_train(epochs - 1, 256, lr) if epochs > 1 else loss0
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    return s, dt, {"trajectory_steps": steps, "dt": dt, "samples": s.learned_info()["samples"],
                   "epochs": epochs, "loss_first_epoch": loss0, "loss_last_epoch": loss,
                   "setup_s": setup_s, "trajectory_s": t_traj, "train_s": t_train}


def _form_record(prefix, dt, infos, steps, warmup):
    med, iqr = _spread(infos)
    i = infos[-1]
    return {f"{prefix}_ms": dt / steps * 1e3, f"{prefix}_timed_solves": steps, f"{prefix}_warmup": warmup,
            f"{prefix}_ms_median": med, f"{prefix}_ms_iqr": iqr, f"{prefix}_iters": i["iters"],
            f"{prefix}_matvecs": i["matvecs"], f"{prefix}_refinements": i["refinements"],
            f"{prefix}_rel_residual": i["rel_residual"], f"{prefix}_init_rel_residual": i["init_rel_residual"],
            f"{prefix}_fallback": i["fallback_used"], f"{prefix}_fp64_cycles": i["fp64_cycles"],
            f"{prefix}_traction64_launches": i["n_traction"], f"{prefix}_fmm_applies": i["fmm_applies"],
            f"{prefix}_near_ms": i["ms_near"]}


def main_bench(args):
    import torch
    from paper_1606_07428_amd import inputs, rbm

    t_start = time.perf_counter()
    w = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = len(w["shape_id"])
    p_up, fmm, _ = WORKLOAD_DEFAULTS.get(args.workload, (0, 0, 4))
    p_up = p_up if args.p_up is None else args.p_up
    fmm = fmm if args.fmm is None else args.fmm
    points = int(n * 2 * w["p"] * (w["p"] + 1))
    _log(f"workload {args.workload}: n={n} p={w['p']} points={points} p_up={p_up} fmm={fmm} "
         f"({time.perf_counter() - t_start:.1f} s)")
    FT = torch.as_tensor(np.asarray(w["FT"], dtype=np.float64), device=dev)
    VW = torch.zeros_like(FT)

    # 1. the learned warm start, trained on the workload's own RK4 trajectory
    sl, dt, learned = _train_on_trajectory(rbm, torch, w, FT, args.tol, args.train_steps, args.epochs, 1e-3,
                                           rbm.MIXED_FP32, p_up=p_up, fmm_order=fmm)
    cen, quat = sl.bodies()
    _log(f"trained on {learned['samples']} samples, loss {learned['loss_first_epoch']:.3e} -> "
         f"{learned['loss_last_epoch']:.3e} ({time.perf_counter() - t_start:.1f} s)")

    # 2a. the subject: precision form + learned guess, K timed solves
    sl.set_guess_mode(rbm.GUESS_LEARNED)
    dtl, infl = _timed(torch, sl, FT, VW, args.steps, args.warmup)
    VWl = VW.cpu().numpy().copy()
    _log(f"mixed + learned: {dtl / args.steps * 1e3:.1f} ms/solve, {infl[-1]['iters']} it, "
         f"fallback {infl[-1]['fallback_used']} ({time.perf_counter() - t_start:.1f} s)")
    # 2b. precision form + block-diagonal guess, same state
    sl.set_guess_mode(rbm.GUESS_BLOCKDIAG)
    dtb, infb = _timed(torch, sl, FT, VW, args.aux_steps, 1)
    VWb = VW.cpu().numpy().copy()
    _log(f"mixed + block-diagonal: {dtb / args.aux_steps * 1e3:.1f} ms/solve, {infb[-1]['iters']} it "
         f"({time.perf_counter() - t_start:.1f} s)")
    sl.close()
    del sl
    torch.cuda.empty_cache()
    # 2c. plain float64 + block-diagonal guess, same state
    t0 = time.perf_counter()
    s64 = rbm.solver_for(w, tol=args.tol, precision=rbm.FP64, guess=rbm.GUESS_BLOCKDIAG, p_up=p_up)
    s64.set_bodies(w["shape_id"], cen, quat)
    torch.cuda.synchronize()
    setup64 = time.perf_counter() - t0
    dt64, inf64 = _timed(torch, s64, FT, VW, args.fp64_steps, 0)
    VW64 = VW.cpu().numpy().copy()
    _log(f"fp64 + block-diagonal: {dt64 / args.fp64_steps * 1e3:.1f} ms/solve, {inf64[-1]['iters']} it "
         f"({time.perf_counter() - t_start:.1f} s)")
    s64.close()
    del s64
    torch.cuda.empty_cache()

    ms_l = dtl / args.steps * 1e3
    ms_64 = dt64 / args.fp64_steps * 1e3
    pairs64 = inf64[-1]["far_pairs"]
    ppl = infl[-1]["pairs_per_launch"]
    # rooflines of the far-sum kernels of the timed learned solves; the largest is the line's
    rooflines = _rooflines(infl, ppl, args.workload)
    ms_trac = sum(i["ms_traction"] for i in infl)
    n_trac = sum(i["n_traction"] for i in infl)
    trac_avg_s = ms_trac / max(n_trac, 1) / 1e3
    vscale = np.abs(VW64).max()
    solve = {"fp64_solve_far_pairs": pairs64, "pairs_per_launch": ppl}
    solve.update(_form_record("mixed_learned", dtl, infl, args.steps, args.warmup))
    solve.update(_form_record("mixed_bd", dtb, infb, args.aux_steps, 1))
    solve.update(_form_record("fp64_bd", dt64, inf64, args.fp64_steps, 0))
    solve.update({
        "speedup_mixed_learned_vs_fp64": ms_64 / ms_l,
        "speedup_mixed_bd_vs_fp64": ms_64 / (dtb / args.aux_steps * 1e3),
        "mixed_learned_vs_fp64_velocity_rel_err": float(np.abs(VWl - VW64).max() / vscale),
        "mixed_bd_vs_fp64_velocity_rel_err": float(np.abs(VWb - VW64).max() / vscale),
        "solves_per_s": args.steps / dtl,
        "matvecs_per_s": sum(i["matvecs"] for i in infl) / dtl,
        "fp64_solves_per_s": args.fp64_steps / dt64,
        "fp64_matvecs_per_s": sum(i["matvecs"] for i in inf64) / dt64,
        "fp64_solve_gpairs_per_s": pairs64 / (ms_64 / 1e3) / 1e9,
        "traction64_gpairs_per_s": ppl / trac_avg_s / 1e9,
        "fp64_setup_s": setup64,
        "near_pairs": infl[-1]["near_pairs"], "fmm_level": infl[-1]["fmm_level"],
    })
    if infl[-1]["fmm_applies"]:
        solve["fmm_apply_ms_avg"] = sum(i["ms_traction32"] for i in infl) / sum(i["n_traction32"] for i in infl)
    result = {
        "metric": METRIC,
        "value": pairs64 / (ms_l / 1e3) / 1e9,
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_l,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "bodies": n, "p": w["p"], "points": points, "tol": args.tol,
                   "step": "precision form (float32 inner sums"
                           + (f" by the fast multipole method of order {fmm}" if fmm else "")
                           + ", float32 preconditioner, float64 refinement residuals) + learned guess",
                   "near_singular_order": p_up,
                   "value": "off-body pairs of the float64 solve / time of the step",
                   "state": f"after {args.train_steps} RK4 steps (trained on their stage solves)"},
        "roofline": rooflines[0] if rooflines else None,
        "roofline_others": rooflines[1:],
        "solve": solve,
        "learned": learned,
    }
    if not args.no_cpu:
        result["cpu_baseline"] = _cpu_baseline(w, args.cpu_budget, max(1, min(16, os.cpu_count() or 1)))
    _log(f"done ({time.perf_counter() - t_start:.1f} s)")
    print(json.dumps(result), flush=True)


def main_learned_experiment(args):
    """Paired comparison along a trajectory: train on the first `train_steps` RK4
    steps, then at each of the next `eval_steps` states solve from both guesses."""
    import torch
    from paper_1606_07428_amd import inputs, rbm

    w = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    FT = torch.as_tensor(np.asarray(w["FT"], dtype=np.float64), device=dev)
    VW = torch.zeros_like(FT)
    prec = {"fp64": rbm.FP64, "fp32": rbm.MIXED_FP32, "bf16": rbm.MIXED_BF16}[args.precision]
    p_up, fmm, _ = WORKLOAD_DEFAULTS.get(args.workload, (0, 0, 4))
    p_up = p_up if args.p_up is None else args.p_up
    fmm = fmm if args.fmm is None else args.fmm
    s, dt, learned = _train_on_trajectory(rbm, torch, w, FT, args.tol, args.train_steps, args.epochs,
                                          1e-3, prec, p_up=p_up, fmm_order=fmm if prec != rbm.FP64 else 0)
    _log(f"trained: {learned}")
    rows = []
    for k in range(args.eval_steps):
        row = {"step": args.train_steps + k}
        for name, g in (("bd", rbm.GUESS_BLOCKDIAG), ("learned", rbm.GUESS_LEARNED)):
            s.set_guess_mode(g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve_dev(FT, VW)
            torch.cuda.synchronize()
            row[name] = {"iters": info["iters"], "ms": (time.perf_counter() - t0) * 1e3,
                         "init_rel_residual": info["init_rel_residual"],
                         "rel_residual": info["rel_residual"], "fallback": info["fallback_used"]}
        rows.append(row)
        _log(json.dumps(row))
        s.set_guess_mode(rbm.GUESS_BLOCKDIAG)
        if args.retrain_every:
            # keep capturing the trajectory's stage solves and fine-tune every few steps
            s.learned_set_capture(True)
        s.step_rk4(dt, FT)
        if args.retrain_every:
            s.learned_set_capture(False)
            if (k + 1) % args.retrain_every == 0:
                t0 = time.perf_counter()
                loss = s.learned_train(args.retrain_epochs, 256, 1e-3)
                torch.cuda.synchronize()
                row["retrain"] = {"loss": loss, "s": time.perf_counter() - t0}
    it_bd = [r["bd"]["iters"] for r in rows]
    it_l = [r["learned"]["iters"] for r in rows]
    print(json.dumps({"experiment": "learned warm start, paired", "workload": args.workload,
                      "precision": args.precision, "tol": args.tol, "training": learned,
                      "retrain_every": args.retrain_every, "retrain_epochs": args.retrain_epochs,
                      "eval_steps": args.eval_steps, "mean_iters_bd": float(np.mean(it_bd)),
                      "mean_iters_learned": float(np.mean(it_l)),
                      "mean_ms_bd": float(np.mean([r["bd"]["ms"] for r in rows])),
                      "mean_ms_learned": float(np.mean([r["learned"]["ms"] for r in rows])),
                      "fallbacks": int(sum(r["learned"]["fallback"] for r in rows)), "rows": rows}),
          flush=True)
    s.close()


def main_compare(args):
    """One configuration, several solver forms, same state: float64 with the
    block-diagonal guess, then GMRES-IR with fp32 and with bf16 preconditioners.
    Velocity differences are stated against the float64 solve."""
    import torch
    from paper_1606_07428_amd import inputs, rbm

    w = inputs.workload(args.workload)
    _log(f"workload {args.workload} generated")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = len(w["shape_id"])
    FT = torch.as_tensor(np.asarray(w["FT"], dtype=np.float64), device=dev)
    VW = torch.zeros_like(FT)
    out = {"experiment": "solver forms", "workload": args.workload, "bodies": n, "p": w["p"],
           "points": int(n * 2 * w["p"] * (w["p"] + 1)), "tol": args.tol, "forms": {}}
    params = None
    if args.learned_from:
        ws = inputs.workload(args.learned_from)
        _log(f"training workload {args.learned_from} generated")
        FTs = torch.as_tensor(np.asarray(ws["FT"], dtype=np.float64), device=dev)
        st, _, learned = _train_on_trajectory(rbm, torch, ws, FTs, args.tol, args.train_steps or 25,
                                              args.epochs, 1e-3, rbm.MIXED_FP32, args.p_up or 0, args.near_factor,
                                              fmm_order=args.fmm or 0)
        params = st.learned_params()
        out["learned_transfer"] = dict(learned, trained_on=args.learned_from)
        st.close()
        del st
        torch.cuda.empty_cache()
        _log(f"trained on {args.learned_from}: {learned}")
    pu = args.p_up or 0
    bd, zero = rbm.GUESS_BLOCKDIAG, rbm.GUESS_ZERO
    forms = [("fp64", rbm.FP64, False, pu, 0, bd), ("mixed_fp32", rbm.MIXED_FP32, False, pu, 0, bd),
             ("mixed_bf16", rbm.MIXED_BF16, False, pu, 0, bd)]
    if params is not None:
        forms.append(("mixed_fp32_learned", rbm.MIXED_FP32, True, pu, 0, bd))
    if args.fmm:
        forms += [("mixed_fp32_fmm", rbm.MIXED_FP32, False, pu, args.fmm, bd),
                  ("mixed_fp32_fmm_zero", rbm.MIXED_FP32, False, pu, args.fmm, zero),
                  ("mixed_bf16_fmm", rbm.MIXED_BF16, False, pu, args.fmm, bd)]
        if params is not None:
            forms.append(("mixed_fp32_fmm_learned", rbm.MIXED_FP32, True, pu, args.fmm, bd))
        out["fmm_order"] = args.fmm
    keep = set(args.forms.split(",")) if args.forms else None
    if keep is not None:
        forms = [f for f in forms if f[0] in keep]
    if pu:
        out["p_up"], out["near_factor"] = pu, args.near_factor
        if keep is None or "fp64_plain" in keep:
            # the plain smooth rule first: the upsampled float64 solve is then the reference
            # (at surface gaps far below the node spacing it may not converge)
            forms.insert(0, ("fp64_plain", rbm.FP64, False, 0, 0, bd))
    ref = None
    plain = None
    for name, prec, use_net, form_pu, fmm_order, guess in forms:
        t0 = time.perf_counter()
        s = rbm.solver_for(w, tol=args.tol, precision=prec, guess=guess, p_up=form_pu,
                           near_factor=args.near_factor, fmm_order=fmm_order)
        if use_net:
            s.learned_bind(k_nbr=8, hidden=256, n_hidden=3, capacity=1, batch_max=1024, seed=7)
            s.learned_set_params(params)
            s.set_guess_mode(rbm.GUESS_LEARNED)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        _log(f"{name}: setup {setup:.2f} s")
        dt, infos = _timed(torch, s, FT, VW, args.steps, args.warmup)
        v = VW.cpu().numpy().copy()
        if form_pu == 0 and pu:
            plain = v
        elif ref is None:
            ref = v
            out["reference_form"] = name
        i = infos[-1]
        out["forms"][name] = {
            "setup_s": setup, "solve_ms": dt / args.steps * 1e3, "iters": i["iters"],
            "matvecs": i["matvecs"], "refinements": i["refinements"], "rel_residual": i["rel_residual"],
            "traction_launch_ms_avg": i["ms_traction"] / max(i["n_traction"], 1),
            "traction32_ms_avg": i["ms_traction32"] / max(i["n_traction32"], 1),
            "n_traction64": i["n_traction"], "n_traction32": i["n_traction32"],
            "stokeslet_ms": i["ms_stokeslet"], "self_ms": i["ms_self"],
            "pairs_per_launch": i["pairs_per_launch"],
            "velocity_rel_err_vs_reference": float(np.abs(v - ref).max() / np.abs(ref).max()) if ref is not None else 0.0,
            "init_rel_residual": i["init_rel_residual"], "fallback": i["fallback_used"],
            "near_pairs": i["near_pairs"], "near_ms": i["ms_near"],
            "fmm_level": i["fmm_level"], "fmm_applies": i["fmm_applies"],
            "workspace_GB": s.workspace_bytes / 1e9}
        if plain is not None and form_pu:
            out["forms"][name]["velocity_change_vs_plain_rule"] = float(np.abs(v - plain).max() / np.abs(plain).max())
        _log(f"{name}: {json.dumps(out['forms'][name])}")
        s.close()
        del s
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# Table 2 of the paper (§4): seconds per time step on one Xeon core with an FMM, for the
# 2 x 2 x n/4 sphere lattice; "Apply" is one application of the operator, "Solve" the GMRES
# solve to 1e-6.  Context only (other hardware, other far-field algorithm).
PAPER_TABLE2 = {(32, 8): (1.09, 10.25), (64, 8): (2.26, 19.51), (128, 8): (4.75, 38.41),
                (32, 16): (10.7, 108.9), (64, 16): (21.5, 220.3), (128, 16): (42.9, 439.9)}


def main_apply(args):
    """Float64 operator applications y = A mu (the matvec of the hot path) at a workload, with
    the near-singular upsampling its solves use: setup, then K timed applications of random
    densities.  Short enough to run under hardware counters."""
    import torch
    from paper_1606_07428_amd import inputs, rbm

    w = inputs.workload(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p_up = WORKLOAD_DEFAULTS.get(args.workload, (0, 0, 4))[0] if args.p_up is None else args.p_up
    s = rbm.solver_for(w, tol=args.tol, precision=rbm.FP64, p_up=p_up)
    mu = torch.randn(3, s.N, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(0))
    s.apply_dev(mu)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.apply_dev(mu)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    N = s.N
    pairs = float(N) * N - float(s.n) * s.M * s.M
    print(json.dumps({"experiment": "float64 operator applications", "workload": args.workload, "points": N,
                      "p_up": p_up, "applications": args.steps, "apply_ms": dt * 1e3,
                      "pairs_per_apply": pairs}), flush=True)
    s.close()


def main_lattice(args):
    """Per-matvec and per-solve times on the paper's sphere lattice (float64, block-diagonal
    guess, tolerance 1e-6 as in the paper), next to the paper's Table 2."""
    import torch
    from paper_1606_07428_amd import inputs, rbm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rows = []
    for (n, p), (apply_s, solve_s) in sorted(PAPER_TABLE2.items(), key=lambda t: (t[0][1], t[0][0])):
        w = inputs.lattice(n, p)
        s = rbm.solver_for(w, tol=1e-6, precision=rbm.FP64, guess=rbm.GUESS_BLOCKDIAG)
        N = n * 2 * p * (p + 1)
        mu = torch.randn(3, N, dtype=torch.float64, device=dev)
        s.apply_dev(mu)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            s.apply_dev(mu)
        torch.cuda.synchronize()
        t_apply = (time.perf_counter() - t0) / reps
        FT = torch.as_tensor(np.asarray(w["FT"]), device=dev)
        VW = torch.zeros_like(FT)
        dt, infos = _timed(torch, s, FT, VW, args.steps, args.warmup)
        row = {"n": n, "p": p, "unknowns": 3 * N, "apply_ms": t_apply * 1e3,
               "solve_ms": dt / args.steps * 1e3, "iters": infos[-1]["iters"],
               "rel_residual": infos[-1]["rel_residual"],
               "paper_apply_s": apply_s, "paper_solve_s": solve_s,
               "apply_ratio_paper_over_ours": apply_s / t_apply,
               "solve_ratio_paper_over_ours": solve_s / (dt / args.steps)}
        _log(json.dumps(row))
        rows.append(row)
        s.close()
        del s
        torch.cuda.empty_cache()
    print(json.dumps({"experiment": "paper lattice (§4, Table 2)", "precision": "fp64", "tol": 1e-6,
                      "rows": rows}), flush=True)


# The paper's magnetorheological run (§4, Fig. 1): 512 paramagnetic spheres on a cubic
# lattice at p = 8, about 5 minutes per time step on one Xeon E5-2690 v2 node with Stokes and
# Laplace FMMs.  Context only.
PAPER_MHD_STEP_S = 300.0


def main_mhd(args):
    """Magnetostatic solve, density-driven mobility solve and one RK4 step of the
    magnetorheological lattice (float64)."""
    import torch
    from paper_1606_07428_amd import inputs, rbm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = inputs.mhd_lattice(side=8, p=8, spacing=args.mhd_spacing, jitter=0.1)
    H0 = 10.0 / math.sqrt(3.0) * np.array([1.0, -1.0, -1.0])
    mu_r = 2.0
    s = rbm.solver_for(w, tol=args.tol, precision=rbm.FP64, guess=rbm.GUESS_BLOCKDIAG, magnetic=1)
    _log(f"mhd: {s.n} bodies, N = {s.N}")
    rho, FT, it = s.magnetic_traction(H0, mu_r, tol=args.tol)
    VW = torch.zeros((s.n, 6), dtype=torch.float64, device=dev)
    s.solve_density_dev(rho, VW)
    torch.cuda.synchronize()
    reps = max(args.steps, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        rho, FT, it = s.magnetic_traction(H0, mu_r, tol=args.tol)
    torch.cuda.synchronize()
    t_mag = (time.perf_counter() - t0) / reps
    _log(f"mhd: magnetostatic solve {t_mag * 1e3:.2f} ms, {it} iterations")
    t0 = time.perf_counter()
    for _ in range(reps):
        info = s.solve_density_dev(rho, VW)
    torch.cuda.synchronize()
    t_mob = (time.perf_counter() - t0) / reps
    _log(f"mhd: mobility solve {t_mob * 1e3:.2f} ms, {info['iters']} iterations")
    vmax = float(VW[:, :3].norm(dim=1).max())
    dt = 0.05 / max(vmax, 1e-12)
    s.step_rk4_magnetic(dt, H0, mu_r, tol_mag=args.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        infos = s.step_rk4_magnetic(dt, H0, mu_r, tol_mag=args.tol)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / reps
    out = {"experiment": "magnetorheological lattice (§4, Fig. 1)", "bodies": s.n, "p": 8,
           "spacing": args.mhd_spacing, "jitter": 0.1, "H0": H0.tolist(), "mu_ratio": mu_r, "tol": args.tol,
           "unknowns_per_step": 4 * s.N, "magnetostatic_ms": t_mag * 1e3, "magnetostatic_iters": it,
           "mobility_ms": t_mob * 1e3, "mobility_iters": info["iters"], "rk4_step_ms": t_step * 1e3,
           "rk4_stage_iters": [i["iters"] for i in infos], "dt": dt, "max_speed": vmax,
           "max_net_force": float(FT[:, :3].norm(dim=1).max()),
           "paper_step_s": PAPER_MHD_STEP_S}
    print(json.dumps(out), flush=True)
    s.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--train-steps", type=int, default=None)
    ap.add_argument("--eval-steps", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--aux-steps", type=int, default=2,
                    help="timed solves of the precision form with the block-diagonal guess")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed plain float64 solves (no warm-up solve)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-experiment", action="store_true")
    ap.add_argument("--compare", action="store_true",
                    help="time fp64 / mixed fp32 / mixed bf16 solves of one workload")
    ap.add_argument("--forms", default=None,
                    help="with --compare: comma list among fp64_plain,fp64,mixed_fp32,mixed_bf16,"
                         "mixed_fp32_learned,mixed_fp32_fmm,mixed_fp32_fmm_zero,mixed_bf16_fmm,"
                         "mixed_fp32_fmm_learned (velocity differences against the first)")
    ap.add_argument("--learned-from", default=None,
                    help="with --compare: train the warm start on this workload's trajectory and "
                         "add a mixed fp32 + learned solve (same p and feature layout)")
    ap.add_argument("--p-up", type=int, default=None,
                    help="near-singular upsampling order (0 = off; default per workload); in compare mode "
                         "a plain-rule float64 reference solve is added")
    ap.add_argument("--near-factor", type=float, default=5.0,
                    help="compare mode: kappa of the near test (mean node spacings)")
    ap.add_argument("--retrain-every", type=int, default=0,
                    help="learned experiment: keep capturing during evaluation and fine-tune the "
                         "network every this many RK4 steps (0 = train once)")
    ap.add_argument("--retrain-epochs", type=int, default=3,
                    help="learned experiment: epochs of each fine-tuning")
    ap.add_argument("--fmm", type=int, default=None,
                    help="fast multipole order of the inner far sums (default per workload); in compare "
                         "mode adds mixed forms whose inner iterations use it")
    ap.add_argument("--apply", action="store_true",
                    help="only time float64 operator applications (y = A mu) at the workload")
    ap.add_argument("--lattice", action="store_true",
                    help="per-matvec and per-solve times on the paper's sphere lattice (Table 2)")
    ap.add_argument("--mhd", action="store_true",
                    help="magnetostatic + mobility solves and RK4 steps of the paper's magnetorheological lattice")
    ap.add_argument("--mhd-spacing", type=float, default=3.0,
                    help="with --mhd: lattice centre spacing (unit spheres)")
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
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path "
              "(bodies sharded across GPUs, sources all-gathered per matvec) is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.apply:
        args.workload = args.workload or "dense4000"
        main_apply(args)
        return
    if args.compare:
        args.workload = args.workload or "ellipsoids1000"
        main_compare(args)
        return
    if args.lattice:
        main_lattice(args)
        return
    if args.mhd:
        main_mhd(args)
        return
    if args.learned_experiment:
        args.workload = args.workload or "sediment512"
        args.train_steps = 25 if args.train_steps is None else args.train_steps
        main_learned_experiment(args)
    else:
        args.workload = args.workload or "dense4000"
        if args.train_steps is None:
            args.train_steps = WORKLOAD_DEFAULTS.get(args.workload, (0, 0, 4))[2]
        main_bench(args)


if __name__ == "__main__":
    main()
