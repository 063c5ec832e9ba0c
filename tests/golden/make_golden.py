"""Write tests/golden/<config>_samples.json from the CPU oracle only.

Configurations (unit square, Neumann; seeded u0 from ``workloads``):
  c2  linearized CH, beta = 0.5, eps = 0.05, 128 x 128 cells, 128 levels, dt = 1e-5  (seconds)
  c3  nonlinear CH (fully implicit backward Euler), eps = 0.01, 256 x 256 cells,
      256 levels, dt = 1e-6, u0 ~ U[-0.1, 0.1]                                       (~2 min)
  c5  nonlinear CH, eps = 0.0075, 512 x 512 cells, 1024 levels, dt = 1e-6,
      u0 ~ U[-0.05, 0.05]                                                            (~1 h)
  c4  the eight smallest requests of the served stream (seed 4): one record each,
      in c4_samples.json under "requests"                                           (seconds)

Stored for every level n = 1..N_t:
  * ||u_n||_2, the discrete mass and the Ginzburg-Landau energy;
  * four projections <w_q, u_n> on seeded standard-normal weight arrays w_q
    (numpy default_rng(PROJ_SEED + q), shape of one level) -- an error anywhere
    in a level moves them by about its own size, so together with the norms
    they check every level of a solve, not only sampled points;
and u_n itself at 256 seeded points for 16 levels.  The full solution (up to
2.1 GB) is not stored.

Run:  python tests/golden/make_golden.py c2|c3|c4|c5
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import operators as ops  # noqa: E402
from oracle import stepper  # noqa: E402
from workloads import CONFIGS, initial_datum, request_u0, served_stream  # noqa: E402

PROJ_SEED = 4321
N_PROJ = 4
N_POINTS = 256


def sample_levels(nt: int):
    """About 16 levels spread over 1..nt (geometric near the start, where the
    solution changes fastest, and uniform), the first and the last included."""
    geo = np.round(np.geomspace(1, nt, 10)).astype(int).tolist()
    lin = np.linspace(1, nt, 8).astype(int).tolist()
    return sorted(set(geo + lin))


def projection_weights(shape):
    return [np.random.default_rng(PROJ_SEED + q).standard_normal(shape) for q in range(N_PROJ)]


def record(p, u0):
    """Stored oracle data of one problem (see the module docstring)."""
    t0 = time.time()
    iters = None
    if p.op == "ch":
        U, iters = stepper.ch_implicit(p.dim, p.n, p.nt, p.dt, u0, p.eps, return_iters=True)
        how = ("sequential backward-Euler CH, banded-Cholesky chord iterations until the increment "
               "and dt ||F||_inf are below 1e-14")
    else:
        U = stepper.sequential(p, u0)
        how = "sequential theta-method, one banded-Cholesky solve per level"
    el = time.time() - t0
    rng = np.random.default_rng(1234)
    pts = rng.integers(0, p.n, size=(N_POINTS, 2))
    levels = sample_levels(p.nt)
    ws = projection_weights(p.slice_shape)
    out = {
        "problem": {"op": p.op, "dim": p.dim, "n": p.n, "nt": p.nt, "dt": p.dt, "eps": p.eps, "beta": p.beta,
                    "theta": p.theta},
        "oracle": how,
        "oracle_seconds": round(el, 1),
        "norms": [float(np.sqrt(np.sum(u * u))) for u in U],
        "mass": [ops.mass(u, p.h) for u in U],
        "energy": [ops.energy(u, p.eps, p.h) for u in U],
        "energy0": ops.energy(u0, p.eps, p.h),
        "mass0": ops.mass(u0, p.h),
        "proj_seed": PROJ_SEED,
        "projections": [[float(np.sum(w * u)) for w in ws] for u in U],
        "points": pts.tolist(),
        "samples": {str(n): [float(U[n - 1][y, x]) for y, x in pts] for n in levels},
    }
    if iters is not None:
        out["chord_iterations_max"] = int(max(iters))
        out["chord_iterations_total"] = int(sum(iters))
    return out


def served_sample(count: int = 8):
    """Indices of the `count` smallest requests of the served stream (seed 4)."""
    reqs = served_stream(n_requests=512, seed=4, rate=1.0)
    dof = np.array([r.problem.dof for r in reqs])
    return reqs, [int(i) for i in np.argsort(dof, kind="stable")[:count]]


def main(name="c3"):
    if name == "c4":
        reqs, idx = served_sample()
        out = {"config": name, "requests": {str(i): record(reqs[i].problem, request_u0(reqs[i])) for i in idx}}
    else:
        out = {"config": name, **record(CONFIGS[name], initial_datum(name))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}")


if __name__ == "__main__":
    main(*(sys.argv[1:]))
