"""Pins of the oracle's all-at-once iteration (CPU only).

* Exact WR error recursion (Section 2.2, fully discrete analysis, eq.
  linear-theta1_err / linear-theta1_err2): per cosine mode with stability
  factor R, every iterate's error is e_n^k = R^n e_0^k with
  e_0^k = alpha (e_{N_t}^k - e_{N_t}^{k-1}), i.e.
  e_0^k = -alpha e_{N_t}^{k-1} / (1 - alpha R^{N_t}).
* The correction form U <- U + P_alpha^{-1} r(U) gives the same iterates as
  the paper's form P_alpha U^k = b^{k-1}.
* The two preconditioner solves (sparse direct, and per-mode dense solves in
  the explicit cosine basis) agree for every operator.
* The linear contraction bound |alpha|/(1-|alpha|) of thm3.
* Converged iterates equal the sequential solution (linear and nonlinear).
"""
import numpy as np
import pytest

from oracle import allatonce as aao
from oracle import stepper
from workloads import Problem


def _modes(E, dim):
    return aao.dct2(E, dim).reshape(E.shape[0], -1)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_exact_wr_error_recursion(theta):
    rng = np.random.default_rng(21)
    p = Problem(op="biharmonic", dim=1, n=8, nt=6, dt=2e-4, theta=theta, alpha=0.2)
    u0 = rng.uniform(-1, 1, 8)
    S = stepper.sequential(p, u0)
    U0 = rng.uniform(-1, 1, p.shape)
    hist = aao.outer_iterate(p, u0, U0, 4, modal=False)
    lam = 2.0 * 64 * (np.cos(np.arange(8) * np.pi / 8) - 1.0)
    z = p.dt * lam ** 2
    R = (1 - (1 - theta) * z) / (1 + theta * z)
    prev_eNt = _modes(U0 - S, 1)[-1]
    for Uk in hist:
        e = _modes(Uk - S, 1)                       # [nt][modes]
        e0 = -p.alpha * prev_eNt / (1 - p.alpha * R ** p.nt)
        expect = (R[None, :] ** np.arange(1, p.nt + 1)[:, None]) * e0[None, :]
        scale = max(np.max(np.abs(e)), 1e-300)
        assert np.max(np.abs(e - expect)) <= 1e-9 * scale + 1e-15
        prev_eNt = e[-1]


def test_thm3_contraction_bound():
    rng = np.random.default_rng(4)
    p = Problem(op="linear_ch", dim=1, n=16, nt=10, dt=1e-4, alpha=0.1, eps=0.05, beta=0.1)
    u0 = rng.uniform(-1, 1, 16)
    S = stepper.sequential(p, u0)
    hist = aao.outer_iterate(p, u0, rng.uniform(-1, 1, p.shape), 5)
    bound = p.alpha / (1 - p.alpha)
    errs = [np.max(np.abs(_modes(U - S, 1))) for U in hist]
    for a, b in zip(errs, errs[1:]):
        assert b <= bound * a * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_correction_form_equals_paper_form(theta):
    rng = np.random.default_rng(7)
    p = Problem(op="linear_ch", dim=2, n=5, nt=6, dt=1e-4, theta=theta, alpha=0.05, eps=0.1, beta=0.4)
    u0 = rng.uniform(-1, 1, (5, 5))
    U0 = rng.uniform(-1, 1, p.shape)
    a = aao.outer_iterate(p, u0, U0, 3, modal=False)
    b = aao.wr_paper_form(p, u0, U0, 3)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) < 1e-11


@pytest.mark.parametrize("op", ["biharmonic", "linear_ch", "ch", "ch_eyre"])
@pytest.mark.parametrize("dim,n,nt", [(1, 9, 7), (2, 4, 6)])
def test_modal_solve_equals_direct_solve(op, dim, n, nt):
    rng = np.random.default_rng(13)
    p = Problem(op=op, dim=dim, n=n, nt=nt, dt=1e-4, theta=1.0 if "ch" == op[:2] else 0.5,
                eps=0.1, beta=0.3, alpha=0.03)
    r = rng.standard_normal(p.shape)
    d1 = aao.precond_solve(p, r, c_bar=0.4)
    d2 = aao.precond_solve_modal(p, r, c_bar=0.4)
    assert np.max(np.abs(d1 - d2)) < 1e-10 * np.max(np.abs(d1))


@pytest.mark.parametrize("op", ["linear_ch", "ch", "ch_eyre"])
def test_converged_iteration_equals_sequential(op):
    rng = np.random.default_rng(17)
    p = Problem(op=op, dim=2, n=8, nt=8, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3)
    u0 = rng.uniform(-0.3, 0.3, (8, 8))
    S = stepper.sequential(p, u0)
    U = np.broadcast_to(u0, p.shape).copy()
    hist = aao.outer_iterate(p, u0, U, 12)
    assert stepper.rel_err(hist[-1], S) < 1e-12


def test_soft_pin_four_iterations_1d_biharmonic():
    # Section 5.1: from a random guess the 1D biharmonic PinT (h = 1/64,
    # alpha = 1e-3) reaches 1e-10 in four iterations, independently of dt.
    rng = np.random.default_rng(1)
    p = Problem(op="biharmonic", dim=1, n=64, nt=100, dt=1e-3, alpha=1e-3)
    u0 = rng.uniform(-1, 1, 64)
    S = stepper.sequential(p, u0)
    hist = aao.outer_iterate(p, u0, rng.uniform(-1, 1, p.shape), 4)
    errs = [stepper.rel_err(U, S) for U in hist]
    assert errs[3] < 1e-10
    assert errs[2] > 1e-10
