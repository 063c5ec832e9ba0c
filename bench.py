"""Throughput benchmark of the all-at-once space-time solve on one MI355X.

One step = one complete solve (every stage of the hot path: FP64 residual +
DCT-II, alpha-circulant time FFT solve, DCT-III + FP64 update, reductions and
stop rule, repeated until the estimated relative error is below 1e-10) of the
largest single-GPU workload: 2D nonlinear Cahn-Hilliard (PinT-I), 512 x 512
cells, 1024 backward-Euler levels, dt = 1e-6, eps = 0.0075,
u0 ~ U[-0.05, 0.05] seeded, inputs resident in HBM; refined mixed precision
(FP64 residual, forward DCT and update; FP32 time solve and inverse DCT) with
alpha = 1e-4.  Plain FP64, the other precisions and the dense matrix-core time
contraction are timed beside it.  The metric is space-time DOF/s = N_s N_t /
solve time; the result is checked against stored data of the CPU FP64
oracle's sequential solution (tests/golden).  ``--config c2|c3`` selects the
smaller workloads.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
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
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}  # dense, MI355X
BF16_ALPHA = 1e-2  # alpha of the BF16 runs (coarser contraction, larger alpha)
# HBM bytes per launch of the dominant kernel from two rocprofv3 counter passes
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors a plain 256 MiB copy gives),
# profiles/c5_fp32_hbm_traffic.md, c2_fp64_hbm_traffic.md, c2_mixed_hbm_traffic.md.
# Valid for the kernel as measured: drop the entry when that kernel changes.
MEASURED_TRAFFIC = {("c5", "fp32", "rows_fwd"): (1022105.6 * 2.0 + 970043.5) * 1024,
                    ("c2", "fp64", "rows_fwd"): (8678.5 * 2.0 + 8272.0) * 1024,
                    ("c2", "mixed", "rows_fwd"): (11533.0 * 2.0 + 10981.3) * 1024}
PREC_DESC = {
    "mixed": "FP64 residual, FP64 forward DCT, FP32 time FFT solve and inverse DCT, FP64 update "
             "(iterative refinement)",
    "fp32": "FP64 residual, FP32 DCTs and time FFT solve, FP64 update (iterative refinement)",
    "fp64": "FP64 throughout",
    "bf16": "FP64 residual and forward DCT, BF16-operand MFMA time contraction (FP32 accumulate), FP32 inverse "
            "DCT, FP64 update",
    "bf16x3": "as bf16 with a two-term BF16 split of both operands (three products)",
    "fp32_norefine": "FP32 residual, transforms and iterate, no refinement (stops on its plateau)",
    "bf16_norefine": "as fp32_norefine with the BF16 dense time contraction",
}

WORKLOADS = {
    "c2": "2D linearized CH u_t = -beta^2 Lap u - eps^2 Lap^2 u, beta=0.5, eps=0.05, unit square, Neumann, "
          "128x128 cells x 128 backward-Euler levels, dt=1e-5, u0 ~ U[-0.05,0.05] (seed 2)",
    "c3": "2D nonlinear CH (PinT-I), f(u)=u^3-u, eps=0.01, unit square, Neumann, 256x256 cells x 256 levels, dt=1e-6, "
          "u0 ~ U[-0.1,0.1] (seed 3)",
    "c5": "2D nonlinear CH (PinT-I), eps=0.0075, unit square, Neumann, 512x512 cells x 1024 levels, dt=1e-6, "
          "u0 ~ U[-0.05,0.05] (seed 5)",
}
# Every workload is checked against stored data of the oracle's sequential
# solution (tests/golden/<config>_samples.json, written by
# tests/golden/make_golden.py from the oracle only): per-level norms and
# random projections at every level, and points at sampled levels.  The
# oracle itself runs here only in the cpu_baseline leg.
GOLDEN = ("c2", "c3", "c5")
# Headline precision and alpha per workload (the other paths are timed
# beside it).  At 128^2 x 128 the FP64 path with alpha = 1e-6 reaches the
# 1e-10 bar in two outer iterations (the small-alpha two-step convergence of
# the linearized CH experiments, Section 5); the FP32 paths cannot use so
# small an alpha, since their rounding error per iteration grows like
# u_32 / alpha.  The nonlinear CH workloads are limited by the scalar averaged
# Jacobian, not alpha; there alpha = 1e-4 saves one (256^2 x 256) to five
# (512^2 x 1024) iterations against 1e-3 while the FP32 rounding term still
# contracts.  At 512^2 x 1024 the FP32 forward transform costs no extra
# iteration (13 in FP32, mixed and FP64 alike: the nonlinearity, not the
# transform's rounding, sets the rate), so the all-FP32 refined path is the
# fastest at the 1e-10 bar.
HEADLINE = {"c2": ("fp64", 1e-6), "c3": ("mixed", 1e-4), "c5": ("fp32", 1e-4)}

# Algorithmic HBM bytes per space-time DOF per launch of each kernel (working
# type W = 4 bytes for the FP32-refined path, 8 for FP64).  Steady iterations:
#   rows_fwd  (residual + x-DCT-II) : read U (8)                      + write S (W)
#   cols_fwd  (y-DCT-II)            : read S (W)                      + write S (W)
#   time      (time FFT solve)      : read S (W)                      + write S (W)
#   cols_inv  (y-DCT-III)           : read S (W)                      + write S (W)
#   rows_inv  (x-DCT-III + update)  : read S (W) + read U (8)         + write U (8)
# The first iteration starts from the broadcast datum: rows_fwd reads only u0
# (N_s values) and rows_inv does not read U; in 2D its residual and spatial
# transform are the same at every level, so rows_fwd and cols_fwd run on level
# 0 only and the time solve reads that level for all N_t.
STAGES = ["rows_fwd", "cols_fwd", "time_solve", "cols_inv", "rows_inv", "finalize"]
KERNEL_NAMES = {"rows_fwd": "k_rows_fwd", "cols_fwd": "k_cols<fwd>", "time_solve": "k_time_solve",
                "cols_inv": "k_cols<inv>", "rows_inv": "k_rows_inv"}


# Mixed precision: the forward transform is FP64 (rows_fwd writes 8 bytes,
# cols_fwd reads 8 and writes 4), the rest FP32.
def algo_bytes_per_dof(precision: str, dim: int = 1, nt: int = 1):
    w = 8 if precision == "fp64" else 4
    wf = 8 if precision in ("fp64", "mixed") else 4
    steady = {"rows_fwd": 8 + wf, "cols_fwd": wf + w, "time_solve": 2 * w, "cols_inv": 2 * w, "rows_inv": w + 16}
    first = dict(steady, rows_fwd=wf, rows_inv=w + 8)
    if dim == 2:
        first.update(rows_fwd=(8 + wf) / nt, cols_fwd=(wf + w) / nt, time_solve=w + w / nt)
    return steady, first


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Levels of the oracle's sequential solve timed by the CPU baseline when a
# whole solve takes minutes or more (about 10-30 s of host work).
CPU_PREFIX_LEVELS = {"c3": 64, "c5": 8}


def cpu_baseline(name: str, min_seconds: float = 10.0):
    """The oracle (sequential FP64 backward Euler with banded Cholesky) timed
    on the host on the same workload: whole solves until min_seconds pass, or
    for the large workloads the first levels of the sequential solve (its
    factorization included), in DOF of the levels solved per second."""
    import numpy as np
    from oracle import stepper
    from workloads import CONFIGS, initial_datum
    p = CONFIGS[name]
    u0 = initial_datum(name)
    levels = CPU_PREFIX_LEVELS.get(name)
    q = dataclasses.replace(p, nt=levels) if levels else p
    reps = 0
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    while True:
        stepper.sequential(q, u0)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or levels:
            break
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    try:
        from threadpoolctl import threadpool_info
        blas = ",".join(f"{d.get('internal_api')}:{d.get('num_threads')}" for d in threadpool_info())
    except Exception:
        blas = "unknown"
    what = (f"the first {levels} of {p.nt} levels of the sequential solve ({q.dof} DOF, one banded Cholesky "
            f"factorization included)" if levels else
            f"{reps} complete sequential solves of the same workload ({p.dof} DOF each)")
    return {
        "value": reps * q.dof / el,
        "unit": "DOF/s",
        "cores": max(1, int(round(cpu / el))),
        "kind": "oracle",
        "sample": f"{what} in {el:.1f} s; host CPU time / wall = {cpu / el:.2f}; os.cpu_count()={os.cpu_count()}; "
                  f"BLAS {blas}",
    }


def golden_deviation(name: str, U) -> dict:
    """Deviation of a GPU result from the stored oracle data of the workload
    (relative to max_n ||u_n^ref||_2; 'rel' <= 1e-10 is the paper's bar)."""
    from tests import _golden
    if not os.path.exists(os.path.join(_golden.GOLDEN_DIR, f"{name}_samples.json")):
        log(f"no stored oracle data for {name}: result not checked")
        return {"rel": None}
    return _golden.compare(U.cpu().numpy() if hasattr(U, "cpu") else U, _golden.load(name))


SERVED = ("c4: 512 Poisson-arrival requests, biharmonic heat / linearized CH 50/50, grids {64^2,128^2,256^2}, "
          "levels {32,64,128}, eps ~ U[0.02,0.08], beta ~ U[0,0.57], dt=1e-5, u0 ~ U[-0.05,0.05] (seed 4)")


def _spin_until(t_target):
    while True:
        d = t_target - time.perf_counter()
        if d <= 0:
            return
        if d > 2e-3:
            time.sleep(d - 1e-3)


def serving_bench(dev, precision, slots, pool_gib, n_requests, oracle_checks, graphs=True, alpha=0.0, light=False):
    """The served stream through the library's serving loop.

    Closed loop: all requests queued at once; the saturation rate is requests
    (and DOF) per second from the first submission to the last completion.
    Open loop: Poisson arrivals at 0.5x and 0.9x that rate, each request
    submitted at its arrival time; latency = completion - scheduled arrival.
    Device-resident requests (u0 and U in HBM, no host copies) unless
    stated; the host-buffer variant is measured once for the PCIe-inclusive
    rate.  light: saturation and 0.5x only, plus the oracle check."""
    import numpy as np
    import torch
    from paper_2304_14021_amd import Server, Solver
    from tests import _golden
    from workloads import request_u0, served_stream

    reqs = served_stream(n_requests=n_requests, seed=4, rate=1.0)
    if alpha:
        reqs = [dataclasses.replace(r, problem=dataclasses.replace(r.problem, alpha=alpha)) for r in reqs]
    u0h = [request_u0(r) for r in reqs]
    u0d = [torch.from_numpy(u).to(dev) for u in u0h]
    Ud = [torch.empty(r.problem.shape, dtype=torch.float64, device=dev) for r in reqs]
    dof = np.array([r.problem.dof for r in reqs], dtype=np.float64)
    base_arr = np.array([r.arrival for r in reqs])
    torch.cuda.synchronize()
    pool = int(pool_gib * (1 << 30))

    def run(srv, rate, host_io=False):
        """rate None: closed loop.  Returns (wall s, latencies ms, reports)."""
        sched = None if rate is None else base_arr / rate
        h0 = srv.stats()["worker_host_seconds"]
        tickets, t_sub = [], []
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if sched is not None:
                _spin_until(t0 + sched[i])
            t_sub.append(time.perf_counter())
            if host_io:
                tickets.append(srv.submit(r.problem, u0h[i], precision=precision))
            else:
                tickets.append(srv.submit_device(r.problem, u0d[i], Ud[i], precision=precision, sync=False))
        t_subs_done = time.perf_counter() - t0
        reps = [srv.wait(t)[1] for t in tickets]
        wall = time.perf_counter() - t0
        for rp in reps:
            rp["_worker_s"] = srv.stats()["worker_host_seconds"] - h0
            rp["_submit_s"] = t_subs_done
            break
        ts = np.array(t_sub) - t0
        late = ts - (sched if sched is not None else ts)
        lat = np.array([rp["ms_total"] for rp in reps]) + late * 1e3
        return wall, lat, reps

    def summary(wall, lat, reps, rate=None):
        its = [rp["iterations"] for rp in reps]
        bad = sum(rp["status"] != 0 for rp in reps)
        d = {"requests": len(reps), "failed": int(bad), "wall_s": wall, "req_per_s": len(reps) / wall,
             "dof_per_s": float(dof.sum()) / wall, "p50_ms": float(np.percentile(lat, 50)),
             "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
             "iterations_mean": float(np.mean(its)), "submit_loop_s": reps[0]["_submit_s"],
             "worker_host_s": reps[0]["_worker_s"]}
        if rate is not None:
            d["arrival_rate_req_per_s"] = rate
        return d

    out = {"workload": SERVED, "precision": PREC_DESC[precision], "alpha": alpha or reqs[0].problem.alpha, "slots": slots, "pool_bytes": pool,
           "graphs": graphs,
           "io": "device-resident (u0 and U in HBM)"}
    with Server(pool, max_active=slots, graphs=graphs, device=dev) as srv:
        run(srv, None)  # warm-up: captures every (slot, shape class) graph once
        w, lat, reps = run(srv, None)
        sat = summary(w, lat, reps)
        out["saturation"] = sat
        log(f"serving saturation: {json.dumps(sat)}")
        for f in ((0.5,) if light else (0.5, 0.9)):
            rate = f * sat["req_per_s"]
            w, lat, reps = run(srv, rate)
            out[f"load_{f}"] = summary(w, lat, reps, rate)
            log(f"serving at {f} x saturation: {json.dumps(out[f'load_{f}'])}")
        st = srv.stats()
        out["server_stats"] = {k: st[k] for k in ("graphs_captured", "graph_updates", "graph_launches",
                                                  "pool_peak", "failed")}
        if not light:
            # PCIe-inclusive: u0 from and U back to host memory, closed loop
            run(srv, None, host_io=True)
            w, lat, reps = run(srv, None, host_io=True)
            out["host_io_saturation"] = summary(w, lat, reps)
    # one request at a time, each timed alone (plan and workspace made
    # beforehand, not timed): what the same stream costs without batching
    solo = 0.0
    for i, r in enumerate([] if light else reqs):
        s = Solver.for_problem(r.problem, precision=precision, device=dev)
        s.solve(u0d[i], Ud[i])
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s.solve(u0d[i], Ud[i])
        torch.cuda.synchronize()
        solo += time.perf_counter() - ts
        del s
    if not light:
        out["one_at_a_time"] = {"dof_per_s": float(dof.sum()) / solo, "req_per_s": len(reqs) / solo,
                                "note": "sum of standalone solve times of the same requests"}
    # served results (a fresh device-resident pass) against stored data of
    # the oracle's sequential solutions of the smallest requests
    errs = []
    g = _golden.load("c4")["requests"]
    with Server(pool, max_active=slots, device=dev) as srv:
        order = [int(i) for i in g][:oracle_checks]
        tk = [(i, srv.submit_device(reqs[i].problem, u0d[i], Ud[i], precision=precision)) for i in order]
        for i, t in tk:
            srv.wait(t)
            errs.append(_golden.compare(Ud[i].cpu().numpy(), g[str(i)])["rel"])
    out["rel_err_vs_oracle_max"] = float(max(errs)) if errs else None
    out["oracle_checked_requests"] = len(errs)
    return out


def shard_bench(dev, name, precision, ranks, solves):
    """Per-iteration kernel times at one rank's share of a P-rank run, on one
    GPU.  The row and column passes are independent per time level, so a rank
    runs them on nt/P levels of the full grid; the time solve is independent
    per spatial mode, so a rank runs it on N_s/P modes over all nt levels (a
    (n/sqrt(P))^2 grid: P a power of 4).  The exchange between the two layouts
    is not run.  Prints one JSON line."""
    import torch
    from paper_2304_14021_amd import Solver
    from workloads import CONFIGS, initial_datum, u0_uniform

    p = CONFIGS[name]
    r = int(round(ranks ** 0.5))
    if ranks < 4 or r * r != ranks or p.nt % ranks or p.n % r or p.dim != 2:
        raise SystemExit(f"--shard needs a 2D workload and a power of 4 that divides nt and n^2 (got {ranks})")
    level_shard = dataclasses.replace(p, nt=p.nt // ranks)
    mode_shard = dataclasses.replace(p, n=p.n // r)
    side = torch.cuda.Stream(device=dev)

    def per_iteration(q, u0_h):
        s = Solver.for_problem(q, precision=precision, device=dev, stage_timing=True)
        u0 = torch.from_numpy(u0_h).to(dev)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            U = torch.empty(q.shape, dtype=torch.float64, device=dev)
            # per-iteration times only: a shard shape need not reach the stop rule
            s.solve(u0, U, raise_on_error=False)
            reps = [s.solve(u0, U, raise_on_error=False)[1] for _ in range(solves)]
        torch.cuda.synchronize()
        its = sum(x["iterations"] for x in reps)
        out = {st: sum(x["ms_stage"][i] for x in reps) / its for i, st in enumerate(STAGES)}
        del s, U
        torch.cuda.empty_cache()
        return out, its / len(reps)

    full, it_full = per_iteration(p, initial_datum(name))
    lev, it_lev = per_iteration(level_shard, initial_datum(name))
    mode, it_mode = per_iteration(mode_shard, u0_uniform((mode_shard.n,) * 2, 0.05, 5))
    stages = {}
    for st in STAGES:
        shard_ms = mode[st] if st == "time_solve" else lev[st]
        stages[st] = {"full_ms": full[st], "full_over_ranks_ms": full[st] / ranks, "shard_ms": shard_ms}
    log(f"{name} {precision}: iterations full {it_full:.1f}, level shard {it_lev:.1f}, mode shard {it_mode:.1f}")
    for st, v in stages.items():
        log(f"  {st:10s} full {v['full_ms'] * 1e3:9.1f} us  full/P {v['full_over_ranks_ms'] * 1e3:8.1f} us  "
            f"shard {v['shard_ms'] * 1e3:8.1f} us")
    print(json.dumps({
        "metric": "per-iteration kernel time at one rank's shard shape (exchange not run)",
        "unit": "ms", "ranks": ranks, "dtype": "f64" if precision == "fp64" else "f64+f32",
        "config": {"workload": WORKLOADS[name], "precision": precision,
                   "level_shard": list(level_shard.shape), "mode_shard": list(mode_shard.shape)},
        "stages": stages}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["mixed", "fp32", "fp64"],
                    help="headline precision (default: fp64 for c2, else mixed)")
    ap.add_argument("--path-steps", type=int, default=5,
                    help="solves per timed loop of the other precision paths (c5; all steps for the others)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    # served requests: FP64 at alpha = 1e-6 (two outer iterations each, as the headline)
    ap.add_argument("--serve-precision", default="fp64", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--serve-alpha", type=float, default=1e-6, help="alpha of every served request (0: the stream's)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-pool-gib", type=float, default=8.0)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-no-graphs", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of a plain device-to-device copy launched before the steps (counter calibration)")
    ap.add_argument("--alpha", type=float, default=0.0,
                    help="alpha of the headline solve (0: the workload's)")
    ap.add_argument("--shard", type=int, default=0,
                    help="time each kernel at one rank's share of a run on this many GPUs (a power of 4) instead")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2304_14021_amd import Solver
    from workloads import CONFIGS, initial_datum

    name = args.config
    p = CONFIGS[name]
    head_prec, head_alpha = HEADLINE.get(name, ("mixed", None))
    if args.precision is not None and args.precision != head_prec:
        head_prec, head_alpha = args.precision, None
    if args.alpha:
        head_alpha = args.alpha
    args.precision = head_prec
    dev = torch.device("cuda:0")
    if args.shard:
        shard_bench(dev, name, args.precision, args.shard, max(1, min(args.steps, 5)))
        return
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

    # every solve runs on a stream of its own: the legacy default stream costs
    # ~5% at this size, and solve graphs need a non-default stream
    side = torch.cuda.Stream(device=dev)

    def run(prec, steps, warmup, timing, time_path="auto", alpha=None, graph=False, strict=True, field=False):
        q = p if alpha is None else dataclasses.replace(p, alpha=alpha)
        s = Solver.for_problem(q, precision=prec, device=dev, stage_timing=timing, time_path=time_path,
                               graph=graph, field_jacobian=field)
        torch.cuda.synchronize()  # u0 and the workspace were made on the default stream
        with torch.cuda.stream(side):
            U = torch.empty(p.shape, dtype=torch.float64, device=dev)
            for _ in range(warmup):
                s.solve(u0, U, raise_on_error=strict)
            torch.cuda.synchronize()
            lat = []
            reps = []
            t0 = time.perf_counter()
            for _ in range(steps):
                ts = time.perf_counter()
                _, rep = s.solve(u0, U, raise_on_error=strict)
                lat.append((time.perf_counter() - ts) * 1e3)
                reps.append(rep)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        del s
        return el, lat, reps, U

    # timed region: K complete solves, no instrumentation
    el, lat, reps, U = run(args.precision, args.steps, args.warmup, False, alpha=head_alpha)
    value = p.dof * args.steps / el
    iters = [r["iterations"] for r in reps]
    dev_g = golden_deviation(name, U)
    err = dev_g["rel"]
    Uh = U.cpu().numpy()
    # invariants of the result (Section 1): the same solve with the report's
    # mass drift and energy monotonicity, outside the timed region
    s_chk = Solver.for_problem(p if head_alpha is None else dataclasses.replace(p, alpha=head_alpha),
                               precision=args.precision, device=dev, invariants=True)
    U_chk, rep_chk = s_chk.solve(u0)
    invariants = {"mass_drift": rep_chk["mass_drift"], "energy_monotone": rep_chk["energy_monotone"],
                  "bitwise_equal_to_timed_result": bool(torch.equal(U_chk, U))}
    del s_chk, U_chk
    log(f"{name} {args.precision}: {args.steps} solves in {el:.3f}s, iterations {sorted(set(iters))}, "
        f"deviation from the stored oracle data {json.dumps(dev_g)}, update history "
        f"{['%.1e' % x for x in reps[-1]['upd_hist']]}, estimate {reps[-1]['est_rel_err']:.1e}; {invariants}")
    # the same K solves again with HIP events recorded on the solve's stream
    # around every kernel launch (per-kernel durations; events add overhead,
    # so this loop is not the headline number)
    el_ev, _, reps, _ = run(args.precision, args.steps, args.warmup, True, alpha=head_alpha)
    iters = [r["iterations"] for r in reps]

    # per-kernel average launch durations from the stage events (recorded on
    # the solve's stream around every launch of the timed region)
    steady, first = algo_bytes_per_dof(args.precision, p.dim, p.nt)
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
    traffic = MEASURED_TRAFFIC.get((name, args.precision, dom))
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS if ach else None,
                "traffic": traffic / 1e9 if traffic is not None else None, "traffic_unit": "GB per launch",
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
        "dtype": {"fp32": "f64+f32", "mixed": "f64+f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{name}: {WORKLOADS[name]}",
                   "precision": PREC_DESC[args.precision],
                   "dof": p.dof, "alpha": reps[-1]["alpha"], "rtol": 1e-10,
                   "iterations": iters[-1]},
        "rel_err_vs_oracle": err,
        "oracle_check": {"kind": "stored oracle data (tests/golden): per-level norms and 4 random projections "
                                 "at every level, 256 points at ~16 levels; each deviation / max_n ||u_n^ref||_2",
                         **dev_g},
        "invariants": invariants,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "roofline": roofline,
        "kernels": kern,
        "finalize_avg_us": kern_fin_us,
        "algo_bytes_per_dof_iteration": sum(steady.values()),
    }
    if not args.no_fp64_compare:
        # the other precision modes and the dense time contraction, same
        # workload and step count (value loop without events; the dense
        # variants get a second loop with events for the contraction kernel)
        out["paths"] = {}
        ps = min(args.steps, args.path_steps) if name == "c5" else args.steps
        pw = min(args.warmup, 1) if name == "c5" else args.warmup
        # the headline path replayed from a captured solve graph (PINT_FLAG_SOLVE_GRAPH)
        elg, _, _, _ = run(args.precision, ps, pw, False, alpha=head_alpha, graph=True)
        out["paths"][f"{args.precision}_solve_graph"] = {"value": p.dof * ps / elg,
                                                         "ms_per_step": elg / ps * 1e3}
        # every refined path at the headline's alpha, then the headline path at
        # the workload's alpha
        variants = [(o, "fft", head_alpha) for o in ("mixed", "fp32", "fp64") if o != args.precision]
        if head_alpha is not None and head_alpha != p.alpha:
            variants += [(args.precision, "fft", p.alpha)]
        variants += [("fp32_norefine", "fft", None)]  # the unrefined plateau (not at the 1e-10 bar)
        if p.op == "ch":
            # the space-varying averaged Jacobian (inner BiCGStab per outer step)
            variants += [(args.precision, "field", head_alpha)]
        # BF16 runs take a larger alpha where admissible (alpha R^{N_t} < 1/2)
        # at 512^2 x 1024 the alpha part of the contraction, alpha R^{N_t} / (1 - alpha R^{N_t}) with
        # R^{N_t} ~ exp(T / (4 eps^2)) ~ 85, is 0.09 at alpha = 1e-3 and 0.5 at 4e-3 (which then does not
        # converge together with the scalar-Jacobian rate); BF16 rounding grows like u_bf16 / alpha
        bf16_alpha = 1e-3 if name == "c5" else BF16_ALPHA
        variants += [("mixed", "dense", None), ("fp32", "dense", None), ("bf16x3", "dense", bf16_alpha),
                     ("bf16", "dense", bf16_alpha), ("bf16_norefine", "dense", bf16_alpha)]
        for prec, tp, al in variants:
            key = prec if tp == "fft" else f"{prec}_{tp}"
            if prec == args.precision and tp == "fft":
                key = f"{prec}_alpha_{al:g}"
            field = tp == "field"
            elo, _, repso, Uo = run(prec, ps, pw, False, "auto" if field else tp, al, strict=False, field=field)
            log(f"{key} status {repso[-1]['status']} update history {['%.1e' % x for x in repso[-1]['upd_hist']]}")
            Uoh = Uo.cpu().numpy()
            d = {"value": p.dof * ps / elo, "ms_per_step": elo / ps * 1e3, "steps": ps,
                 "status": repso[-1]["status"], "iterations": repso[-1]["iterations"], "alpha": repso[-1]["alpha"],
                 **({"inner_iterations": repso[-1]["inner_iterations"]} if field else {}),
                 "rel_err_vs_oracle": golden_deviation(name, Uoh)["rel"],
                 "rel_diff_vs_headline": float(np.max(np.sqrt(np.sum((Uoh - Uh).reshape(p.nt, -1) ** 2, axis=1)))
                                               / np.max(np.sqrt(np.sum(Uh.reshape(p.nt, -1) ** 2, axis=1))))}
            del Uo, Uoh
            if tp == "dense":
                _, _, repe, _ = run(prec, ps, pw, True, tp, al, strict=False)
                its = sum(r["iterations"] for r in repe)
                us = sum(r["ms_stage"][2] for r in repe) / max(1, its) * 1e3
                flops = 4.0 * p.nt * p.dof * (3 if prec == "bf16x3" else 1)
                peak = MFMA_PEAK_TFLOPS["bf16" if prec.startswith("bf16") else "fp32"]
                ach = flops / (us * 1e-6) / 1e12
                d["time_contraction"] = {"bound": "mfma", "kernel": "k_time_dense", "avg_launch_us": us,
                                         "flops_per_launch": flops, "achieved": ach, "peak": peak,
                                         "unit": "TFLOP/s", "frac": ach / peak,
                                         "hbm_gbs": 8.0 * p.dof / (us * 1e-6) / 1e9}
                log(f"{key}: contraction {us:.1f} us, {ach:.1f} TFLOP/s ({100 * ach / peak:.1f}% of {peak})")
            out["paths"][key] = d
    if not args.no_serving:
        out["serving"] = serving_bench(dev, args.serve_precision, args.serve_slots, args.serve_pool_gib,
                                       args.serve_requests, oracle_checks=8, graphs=not args.serve_no_graphs,
                                       alpha=args.serve_alpha)
        # the same stream in the other precision (FP64 <-> refined mixed)
        alt = "mixed" if args.serve_precision == "fp64" else "fp64"
        out["serving_" + alt] = serving_bench(dev, alt, args.serve_slots, args.serve_pool_gib, args.serve_requests,
                                              oracle_checks=8, graphs=not args.serve_no_graphs,
                                              alpha=args.serve_alpha, light=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
