"""Throughput benchmark of the all-at-once space-time solve on one MI355X.

One step = one complete solve (every stage of the hot path: FP64 residual +
DCT-II, alpha-circulant time FFT solve, DCT-III + FP64 update, reductions and
stop rule, repeated until the estimated relative error is below 1e-10) of the
2D linearized Cahn-Hilliard workload (128 x 128 cells, 128 backward-Euler
levels, dt = 1e-5, beta = 0.5, eps = 0.05, u0 ~ U[-0.05, 0.05] seeded),
inputs resident in HBM.  The metric is space-time DOF/s = N_s N_t / solve time,
with the result checked against the CPU FP64 oracle.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "space-time DOF/s at 1e-10 rel err vs FP64 oracle; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
PREC_DESC = {
    "mixed": "FP64 residual, FP64 forward DCT, FP32 time FFT solve and inverse DCT, FP64 update "
             "(iterative refinement)",
    "fp32": "FP64 residual, FP32 DCTs and time FFT solve, FP64 update (iterative refinement)",
    "fp64": "FP64 throughout",
}

WORKLOADS = {
    "c2": "2D linearized CH u_t = -beta^2 Lap u - eps^2 Lap^2 u, beta=0.5, eps=0.05, unit square, Neumann, "
          "128x128 cells x 128 backward-Euler levels, dt=1e-5, u0 ~ U[-0.05,0.05] (seed 2)",
    "c1": "1D biharmonic heat, 64 cells x 32 backward-Euler levels, T=1e-3, u0=cos(pi x)+0.5cos(3 pi x)+1e-3 N(0,1)",
}

# Algorithmic HBM bytes per space-time DOF per launch of each kernel (working
# type W = 4 bytes for the FP32-refined path, 8 for FP64).  Steady iterations:
#   rows_fwd  (residual + x-DCT-II) : read U (8)                      + write S (W)
#   cols_fwd  (y-DCT-II)            : read S (W)                      + write S (W)
#   time      (time FFT solve)      : read S (W)                      + write S (W)
#   cols_inv  (y-DCT-III)           : read S (W)                      + write S (W)
#   rows_inv  (x-DCT-III + update)  : read S (W) + read U (8)         + write U (8)
# The first iteration starts from the broadcast datum: rows_fwd reads only u0
# (N_s values) and rows_inv does not read U.
STAGES = ["rows_fwd", "cols_fwd", "time_solve", "cols_inv", "rows_inv", "finalize"]
KERNEL_NAMES = {"rows_fwd": "k_rows_fwd", "cols_fwd": "k_cols<fwd>", "time_solve": "k_time_solve",
                "cols_inv": "k_cols<inv>", "rows_inv": "k_rows_inv"}


# Mixed precision: the forward transform is FP64 (rows_fwd writes 8 bytes,
# cols_fwd reads 8 and writes 4), the rest FP32.
def algo_bytes_per_dof(precision: str):
    w = 8 if precision == "fp64" else 4
    wf = 8 if precision in ("fp64", "mixed") else 4
    steady = {"rows_fwd": 8 + wf, "cols_fwd": wf + w, "time_solve": 2 * w, "cols_inv": 2 * w, "rows_inv": w + 16}
    first = dict(steady, rows_fwd=wf, rows_inv=w + 8)
    return steady, first


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(name: str, min_seconds: float = 10.0):
    """The oracle (sequential FP64 backward Euler with banded Cholesky) timed
    on the host on whole solves of the same workload until min_seconds pass."""
    import numpy as np
    from oracle import stepper
    from workloads import CONFIGS, initial_datum
    p = CONFIGS[name]
    u0 = initial_datum(name)
    reps = 0
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    while True:
        stepper.sequential(p, u0)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    try:
        from threadpoolctl import threadpool_info
        blas = ",".join(f"{d.get('internal_api')}:{d.get('num_threads')}" for d in threadpool_info())
    except Exception:
        blas = "unknown"
    return {
        "value": reps * p.dof / el,
        "unit": "DOF/s",
        "cores": max(1, int(round(cpu / el))),
        "kind": "oracle",
        "sample": f"{reps} complete sequential solves of the same workload ({p.dof} DOF each) in {el:.1f} s; "
                  f"host CPU time / wall = {cpu / el:.2f}; os.cpu_count()={os.cpu_count()}; BLAS {blas}",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of a plain device-to-device copy launched before the steps (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from oracle import stepper
    from paper_2304_14021_amd import Solver
    from workloads import CONFIGS, initial_datum

    name = args.config
    p = CONFIGS[name]
    dev = torch.device("cuda:0")
    u0_h = initial_datum(name)
    u0 = torch.from_numpy(u0_h).to(dev)

    if args.calibrate_copy:
        nb = args.calibrate_copy // 4
        a = torch.ones(nb, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb * 4} bytes read, {nb * 4} bytes written")
        del a, b

    def run(prec, steps, warmup, timing):
        s = Solver.for_problem(p, precision=prec, device=dev, stage_timing=timing)
        U = torch.empty(p.shape, dtype=torch.float64, device=dev)
        for _ in range(warmup):
            s.solve(u0, U)
        torch.cuda.synchronize()
        lat = []
        reps = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            _, rep = s.solve(u0, U)
            lat.append((time.perf_counter() - ts) * 1e3)
            reps.append(rep)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return el, lat, reps, U

    # timed region: K complete solves, no instrumentation
    el, lat, reps, U = run(args.precision, args.steps, args.warmup, False)
    value = p.dof * args.steps / el
    iters = [r["iterations"] for r in reps]
    ref = stepper.sequential(p, u0_h)
    err = stepper.rel_err(U.cpu().numpy(), ref)
    log(f"{name} {args.precision}: {args.steps} solves in {el:.3f}s, iterations {sorted(set(iters))}, "
        f"rel err vs oracle {err:.2e}, update history {['%.1e' % x for x in reps[-1]['upd_hist']]}, "
        f"estimate {reps[-1]['est_rel_err']:.1e}")
    # the same K solves again with HIP events recorded on the solve's stream
    # around every kernel launch (per-kernel durations; events add overhead,
    # so this loop is not the headline number)
    el_ev, _, reps, _ = run(args.precision, args.steps, args.warmup, True)
    iters = [r["iterations"] for r in reps]

    # per-kernel average launch durations from the stage events (recorded on
    # the solve's stream around every launch of the timed region)
    steady, first = algo_bytes_per_dof(args.precision)
    tot_iters = sum(iters)
    avg_ms = {}
    for i, st in enumerate(STAGES):
        avg_ms[st] = sum(r["ms_stage"][i] for r in reps) / max(1, tot_iters)
    kern = {}
    for k in steady:
        # average algorithmic bytes per launch over all launches of the region
        per_launch = (first[k] + steady[k] * (tot_iters / len(reps) - 1)) / (tot_iters / len(reps)) * p.dof
        kern[k] = {"avg_us": avg_ms[k] * 1e3, "algo_bytes": per_launch,
                   "gbs": per_launch / (avg_ms[k] * 1e-3) / 1e9 if avg_ms[k] > 0 else None}
    kern_fin_us = avg_ms["finalize"] * 1e3
    dom = max(steady, key=lambda k: avg_ms[k])
    ach = kern[dom]["gbs"]
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": None,
                "kernel": KERNEL_NAMES[dom], "algo_bytes_per_launch": kern[dom]["algo_bytes"],
                "avg_launch_us": kern[dom]["avg_us"]}
    log("kernels: " + json.dumps(kern))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "ms_per_step_with_kernel_events": el_ev / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "mixed": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{name}: {WORKLOADS[name]}",
                   "precision": PREC_DESC[args.precision],
                   "dof": p.dof, "alpha": reps[-1]["alpha"], "rtol": 1e-10,
                   "iterations": iters[-1]},
        "rel_err_vs_oracle": err,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "roofline": roofline,
        "kernels": kern,
        "finalize_avg_us": kern_fin_us,
        "algo_bytes_per_dof_iteration": sum(steady.values()),
    }
    if not args.no_fp64_compare:
        # the other precision modes, same workload and step count (not timed with events)
        out["paths"] = {}
        for other in ("mixed", "fp32", "fp64"):
            if other == args.precision:
                continue
            elo, _, repso, Uo = run(other, args.steps, args.warmup, False)
            log(f"{other} update history {['%.1e' % x for x in repso[-1]['upd_hist']]}")
            out["paths"][other] = {"value": p.dof * args.steps / elo, "ms_per_step": elo / args.steps * 1e3,
                                   "iterations": repso[-1]["iterations"],
                                   "rel_err_vs_oracle": stepper.rel_err(Uo.cpu().numpy(), ref)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
