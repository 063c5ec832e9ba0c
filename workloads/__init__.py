"""Seeded synthetic workloads for the all-at-once space-time solve.

This module only draws inputs (initial data, problem parameters, arrival
times).  It holds none of the method's arithmetic: no operator, no time
stepping, no transform.  Both the CPU oracle (``oracle/``) and the HIP path
(``paper_2304_14021_amd``) are fed from here, so the two sides see the same
FP64 arrays.

The problems follow the paper's model equations with homogeneous Neumann
conditions on the unit interval / unit square (Sections 2-4): the biharmonic
heat equation, the linearized Cahn-Hilliard (CH) equation and the nonlinear CH
equation with f(u) = u^3 - u.  The grid is cell-centred: N cells per
dimension, h = 1/N, x_j = (j + 1/2) h.  The arrays are row-major ``[y][x]``;
a space-time state is ``[N_t][N_y][N_x]`` and holds u_1 .. u_{N_t}
(u_0 is the initial datum, passed separately).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

OPS = ("biharmonic", "linear_ch", "ch", "ch_eyre")


@dataclasses.dataclass(frozen=True)
class Problem:
    """Statement of one all-at-once solve (the paper's problem data).

    op     -- "biharmonic" (u_t = -Lap^2 u), "linear_ch" (u_t = -beta^2 Lap u -
              eps^2 Lap^2 u), "ch" (u_t = Lap(u^3 - u) - eps^2 Lap^2 u, fully
              implicit backward Euler) or "ch_eyre" (convex/concave split).
    dim    -- 1 or 2; n cells per dimension on the unit interval / square.
    nt     -- number of unknown time levels u_1..u_nt; T = nt * dt.
    theta  -- theta-method parameter (1 = backward Euler, 1/2 = trapezoidal).
    q      -- growth ratio of the time steps: dt_n = dt q^(n-1), n = 1..nt
              (1 = uniform steps; see ``time_steps``).
    """

    op: str
    dim: int
    n: int
    nt: int
    dt: float
    theta: float = 1.0
    eps: float = 1.0
    beta: float = 0.0
    alpha: float = 1e-3
    q: float = 1.0

    @property
    def ns(self) -> int:
        return self.n ** self.dim

    @property
    def dof(self) -> int:
        return self.ns * self.nt

    @property
    def h(self) -> float:
        return 1.0 / self.n

    @property
    def shape(self):
        return (self.nt,) + (self.n,) * self.dim

    @property
    def slice_shape(self):
        return (self.n,) * self.dim


def time_steps(p: Problem) -> np.ndarray:
    """The N_t time steps dt_n = dt q^(n-1) of a problem (a geometric grading
    for q > 1, uniform for q = 1), FP64.  Both the oracle and the HIP path
    take the steps from here."""
    return p.dt * p.q ** np.arange(p.nt, dtype=np.float64)


def cell_centres(n: int) -> np.ndarray:
    """x_j = (j + 1/2)/n, j = 0..n-1 (cell-centred grid on (0, 1))."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def u0_c1(n: int = 64, seed: int = 1, noise: float = 1e-3) -> np.ndarray:
    """1D biharmonic initial datum: cos(pi x) + 0.5 cos(3 pi x) + noise*N(0,1)."""
    x = cell_centres(n)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    return np.cos(np.pi * x) + 0.5 * np.cos(3.0 * np.pi * x) + noise * z


def u0_uniform(shape, amp: float, seed: int) -> np.ndarray:
    """i.i.d. uniform[-amp, amp] initial datum (the paper's 0.1*rand[-1,1] kind)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=shape)


# Named configurations.  "c1" is the small case the oracle finishes in
# milliseconds; "c2" is the throughput workload; "c3"/"c5" the nonlinear CH
# cases; "c4" the served stream (see ``served_stream``).
CONFIGS: Dict[str, Problem] = {
    "c1": Problem(op="biharmonic", dim=1, n=64, nt=32, dt=1e-3 / 32, alpha=1e-3),
    "c2": Problem(op="linear_ch", dim=2, n=128, nt=128, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3),
    "c3": Problem(op="ch", dim=2, n=256, nt=256, dt=1e-6, eps=0.01, alpha=1e-3),
    "c5": Problem(op="ch", dim=2, n=512, nt=1024, dt=1e-6, eps=0.0075, alpha=1e-3),
    # geometrically graded steps (1e-6 growing by 1.2 per level, T = 0.58):
    # the time-step matrix is no longer alpha-circulant and is diagonalized
    # directly (FP64 eigendecomposition, dense contraction on the matrix cores)
    "c2g": Problem(op="linear_ch", dim=2, n=128, nt=64, dt=5e-8, eps=0.05, beta=0.5, alpha=0.0, q=1.2),
}

SEEDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5, "c2g": 6}
U0_AMP = {"c2": 0.05, "c3": 0.1, "c5": 0.05, "c2g": 0.05}


def initial_datum(name: str) -> np.ndarray:
    """The seeded FP64 initial datum of a named configuration."""
    p = CONFIGS[name]
    if name == "c1":
        return u0_c1(p.n, SEEDS[name])
    return u0_uniform(p.slice_shape, U0_AMP[name], SEEDS[name])


def small_problem(op: str, dim: int, n: int, nt: int, dt: float, **kw) -> Problem:
    return Problem(op=op, dim=dim, n=n, nt=nt, dt=dt, **kw)


@dataclasses.dataclass(frozen=True)
class Request:
    arrival: float  # seconds after stream start (at the unit rate; scaled by the caller)
    problem: Problem
    seed: int


def served_stream(n_requests: int = 512, seed: int = 4, rate: float = 1.0,
                  grids=(64, 128, 256), nts=(32, 64, 128)) -> List[Request]:
    """Poisson-arrival mix of biharmonic and linearized CH requests.

    Operators 50/50, grid from ``grids`` (2D), time levels from ``nts``,
    eps ~ U[0.02, 0.08], beta ~ U[0, 0.57] (the spinodal range of the
    linearized CH equation is |beta| <= 1/sqrt(3)), dt = 1e-5, and
    u0 ~ U[-0.05, 0.05] drawn from a per-request seed.  ``rate`` is the
    arrival rate in requests per second.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        op = "biharmonic" if rng.random() < 0.5 else "linear_ch"
        n = int(rng.choice(grids))
        nt = int(rng.choice(nts))
        eps = float(rng.uniform(0.02, 0.08))
        beta = float(rng.uniform(0.0, 0.57))
        if op == "biharmonic":
            eps, beta = 1.0, 0.0
        p = Problem(op=op, dim=2, n=n, nt=nt, dt=1e-5, eps=eps, beta=beta, alpha=1e-3)
        out.append(Request(arrival=t, problem=p, seed=1000 + i))
    return out


def request_u0(req: Request) -> np.ndarray:
    return u0_uniform(req.problem.slice_shape, 0.05, req.seed)


def random_guess(p: Problem, seed: int, amp: float = 1.0) -> np.ndarray:
    """A seeded random initial guess for the whole space-time state (the
    paper starts its iterations from a random guess)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=p.shape)
