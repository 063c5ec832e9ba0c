"""Nonuniform time steps: direct diagonalization of the time-step pencil
(Section 1: diagonalization with variable steps; Section 2.1 for the
theta-method blocks), FP64 eigendecomposition on the GPU, dense contraction
time solve, FP64 refinement.

Pins:
  * the plan's eigendecomposition B V = C V diag(d), W C V = I, unit columns,
    d = 1/(theta dt) (brute force in FP64 numpy, and against LAPACK's
    eigenvectors up to sign);
  * the time-solve stage against the oracle's per-mode dense solve
    (B + shift_k C) y = x, no eigendecomposition;
  * whole solves against the sequential oracle with the same steps, both of
    the paper's error norms within 1e-10 (Section 5).
Tolerance of the stage: rounding u of the contraction's working precision
amplified by cond(V) (the refinement loop removes it).
"""
import numpy as np
import pytest
import torch

from oracle import allatonce as aao
from oracle import stepper
from paper_2304_14021_amd import Solver
from workloads import CONFIGS, Problem, initial_datum, time_steps
from tests._gpu import dev, host, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-10

CASES = [
    CONFIGS["c2g"],                                                                   # linear CH 128^2 x 64, q 1.2
    Problem(op="biharmonic", dim=2, n=32, nt=32, dt=1e-6, theta=0.5, q=1.5),          # trapezoidal
    Problem(op="ch", dim=2, n=64, nt=32, dt=1e-6, eps=0.05, q=1.25),                  # nonlinear CH
    Problem(op="linear_ch", dim=1, n=256, nt=64, dt=1e-7, eps=0.05, beta=0.5, q=1.2),
]
IDS = [f"{p.op}-{p.dim}d-n{p.n}-nt{p.nt}-th{p.theta}-q{p.q}" for p in CASES]


def _pencil(dts, theta):
    nt = dts.size
    B = (np.eye(nt) - np.eye(nt, k=-1)) / dts[:, None]
    C = theta * np.eye(nt) + (1.0 - theta) * np.eye(nt, k=-1)
    return B, C


@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_time_step_eigendecomposition(p):
    dts = time_steps(p)
    s = Solver.for_problem(p, precision="fp64", dts=dts, device=dev())
    V, W, d = s.time_eig()
    B, C = _pencil(dts, p.theta)
    cond = np.linalg.cond(V)
    say(f"  {p.op} nt {p.nt} q {p.q} theta {p.theta}: cond(V) {cond:.2e}")
    assert np.array_equal(d, 1.0 / (p.theta * dts))
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, rtol=0, atol=1e-14)
    # B V = C V D, relative to |B| |V|
    res = np.abs(B @ V - C @ V * d[None, :])
    assert np.max(res) <= 1e-13 * np.max(np.abs(B)) * np.max(np.abs(V))
    # biorthogonality W C V = I
    assert np.max(np.abs(W @ C @ V - np.eye(p.nt))) <= 1e-15 * cond * p.nt
    # LAPACK's eigenvectors of C^{-1} B, matched by eigenvalue, up to sign
    lw, lv = np.linalg.eig(np.linalg.solve(C, B))
    lw, lv = np.real(lw), np.real(lv)
    order = np.argsort(lw)
    mine = np.argsort(d)
    assert np.allclose(lw[order], d[mine], rtol=1e-12, atol=0)
    for a, b in zip(order, mine):
        sgn = np.sign(lv[:, a] @ V[:, b])
        assert np.max(np.abs(sgn * lv[:, a] - V[:, b])) <= 1e-15 * cond * p.nt


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_direct_time_solve_stage(p, prec):
    dts = time_steps(p)
    s = Solver.for_problem(p, precision=prec, dts=dts, device=dev())
    rng = np.random.default_rng(41)
    x = rng.standard_normal(p.shape)
    c_bar = 0.37 if p.op == "ch" else 0.0
    wdt = torch.float64 if prec == "fp64" else torch.float32
    y = host(s.time_solve(to_dev(x, dtype=wdt), c_bar)).astype(np.float64)
    ref = aao.time_solve_steps_modal(p, x, dts, c_bar)
    V, _, _ = s.time_eig()
    u = 2.0 ** -52 if prec == "fp64" else 2.0 ** -23
    bound = 16 * u * np.linalg.cond(V) * np.sqrt(p.nt)
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    say(f"  {prec}: stage error {err:.2e} (bound {bound:.2e})")
    assert err <= bound


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp32"])
@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_direct_solve_matches_oracle(p, prec):
    dts = time_steps(p)
    u0 = initial_datum("c2g") if p == CONFIGS["c2g"] else np.random.default_rng(43).uniform(
        -0.1, 0.1, p.slice_shape)
    s = Solver.for_problem(p, precision=prec, dts=dts, device=dev(), invariants=True)
    Ud, rep = s.solve(to_dev(u0), raise_on_error=False)
    U = host(Ud)
    ref = stepper.sequential(p, u0, dts)
    err, err_inf = stepper.rel_err(U, ref), stepper.rel_err_inf(U, ref)
    say(f"  {prec}: status {rep['status']} iterations {rep['iterations']} err {err:.2e} err_inf {err_inf:.2e} "
        f"updates {['%.1e' % v for v in rep['upd_hist']]} mass drift {rep['mass_drift']:.1e}")
    assert rep["status"] == 0
    assert err <= TOL and err_inf <= TOL
    assert rep["mass_drift"] <= 1e-12
