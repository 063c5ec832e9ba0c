"""Write tests/golden/c3_samples.json from the CPU oracle only.

Configuration: 2D nonlinear CH (fully implicit backward Euler), eps = 0.01,
256 x 256 cells on the unit square, 256 levels, dt = 1e-6, u0 ~ U[-0.1, 0.1]
(seed 3).  Stored: per-level ||u_n||_2, mass and Ginzburg-Landau energy, and
u_n at 64 seeded sample points for 8 levels.  The full solution (134 MB) is
not stored; tests compare the GPU solve against these samples.

Run:  python tests/golden/make_golden.py   (about 3 minutes on one core)
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
from workloads import CONFIGS, initial_datum  # noqa: E402

LEVELS = [1, 2, 8, 32, 64, 128, 200, 256]


def main(name="c3"):
    p = CONFIGS[name]
    u0 = initial_datum(name)
    t0 = time.time()
    U, iters = stepper.ch_implicit(p.dim, p.n, p.nt, p.dt, u0, p.eps, return_iters=True)
    el = time.time() - t0
    rng = np.random.default_rng(1234)
    pts = rng.integers(0, p.n, size=(64, 2))
    out = {
        "config": name,
        "problem": {"op": p.op, "dim": p.dim, "n": p.n, "nt": p.nt, "dt": p.dt, "eps": p.eps},
        "oracle": "sequential backward-Euler CH, banded-Cholesky chord iterations to 1e-14",
        "oracle_seconds": round(el, 1),
        "chord_iterations_max": int(max(iters)),
        "norms": [float(np.sqrt(np.sum(u * u))) for u in U],
        "mass": [ops.mass(u, p.h) for u in U],
        "energy": [ops.energy(u, p.eps, p.h) for u in U],
        "energy0": ops.energy(u0, p.eps, p.h),
        "mass0": ops.mass(u0, p.h),
        "points": pts.tolist(),
        "samples": {str(n): [float(U[n - 1][y, x]) for y, x in pts] for n in LEVELS},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_samples.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path} ({el:.0f} s oracle)")


if __name__ == "__main__":
    main(*(sys.argv[1:]))
