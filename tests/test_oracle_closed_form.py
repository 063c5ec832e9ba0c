"""Closed-form pins of the sequential oracle (CPU only).

A cosine mode sampled at the cell centres is an exact eigenvector of the
cell-centred Neumann Laplacian with eigenvalue (2/h^2)(cos(k pi/N) - 1), so
under the theta-method it is multiplied per step by the stability function
R_theta(dt mu_k) of Section 2.2 (eq. linear-theta1_err2): 1/(1 + z) for
backward Euler and (1 - z/2)/(1 + z/2) for the trapezoidal rule, z = dt mu_k.
The expected values below are computed from these formulas alone.
"""
import numpy as np
import pytest

from oracle import stepper
from workloads import CONFIGS, cell_centres


def _lam(k, n):
    h = 1.0 / n
    return 2.0 / h ** 2 * (np.cos(k * np.pi / n) - 1.0)


def _r(theta, z):
    return (1.0 - (1.0 - theta) * z) / (1.0 + theta * z)


def test_c1_noise_free_modes_decay_exactly():
    p = CONFIGS["c1"]
    x = cell_centres(p.n)
    u0 = np.cos(np.pi * x) + 0.5 * np.cos(3 * np.pi * x)
    U = stepper.theta_method("biharmonic", 1, p.n, p.nt, p.dt, u0)
    mu1, mu3 = _lam(1, p.n) ** 2, _lam(3, p.n) ** 2
    # closed-form values at h = 1/64, dt = 1e-3/32, n = 32 steps
    assert abs(mu1 - 97.36997907630963) < 1e-9
    assert abs(mu3 - 7861.664941310234) < 1e-7
    assert abs((1 + p.dt * mu1) ** -32 - 0.907354424362995) < 1e-14
    assert abs((1 + p.dt * mu3) ** -32 - 8.851673924234474e-4) < 1e-16
    n = np.arange(1, p.nt + 1)[:, None]
    exact = (1 + p.dt * mu1) ** (-n) * np.cos(np.pi * x) + 0.5 * (1 + p.dt * mu3) ** (-n) * np.cos(3 * np.pi * x)
    # rounding bound: nt steps x cond(I + dt A) (= 1 + dt mu_max ~ 8.4e3) x 2^-53
    assert np.max(np.abs(U - exact)) < p.nt * (1 + p.dt * _lam(p.n - 1, p.n) ** 2) * 2.2e-16


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("op,eps,beta", [("biharmonic", 1.0, 0.0), ("linear_ch", 0.05, 0.5)])
def test_2d_product_mode(theta, op, eps, beta):
    n, nt, dt = 16, 12, 2e-5
    x = cell_centres(n)
    kx, ky = 2, 3
    u0 = np.outer(np.cos(ky * np.pi * x), np.cos(kx * np.pi * x))  # [y][x]
    U = stepper.theta_method(op, 2, n, nt, dt, u0, theta=theta, eps=eps, beta=beta)
    lam = _lam(kx, n) + _lam(ky, n)
    mu = lam * lam if op == "biharmonic" else beta ** 2 * lam + eps ** 2 * lam * lam
    fac = _r(theta, dt * mu) ** np.arange(1, nt + 1)
    exact = fac[:, None, None] * u0[None]
    assert np.max(np.abs(U - exact)) < 1e-13


def test_spinodal_mode_grows():
    # the linearized CH operator has negative eigenvalues: such a mode grows
    n, nt, dt, eps, beta = 32, 10, 1e-4, 0.05, 0.5
    x = cell_centres(n)
    k = 2
    u0 = np.cos(k * np.pi * x)
    lam = _lam(k, n)
    mu = beta ** 2 * lam + eps ** 2 * lam ** 2
    assert mu < 0
    U = stepper.theta_method("linear_ch", 1, n, nt, dt, u0, eps=eps, beta=beta)
    fac = (1 + dt * mu) ** -np.arange(1, nt + 1)
    assert np.max(np.abs(U - fac[:, None] * u0)) < 1e-13
    assert fac[-1] > 1.0


def test_c1_noisy_case_by_linearity():
    from workloads import u0_c1
    p = CONFIGS["c1"]
    x = cell_centres(p.n)
    smooth = np.cos(np.pi * x) + 0.5 * np.cos(3 * np.pi * x)
    u0 = u0_c1(p.n, 1)
    U = stepper.theta_method("biharmonic", 1, p.n, p.nt, p.dt, u0)
    Un = stepper.theta_method("biharmonic", 1, p.n, p.nt, p.dt, u0 - smooth)
    n = np.arange(1, p.nt + 1)[:, None]
    mu1, mu3 = _lam(1, p.n) ** 2, _lam(3, p.n) ** 2
    exact = (1 + p.dt * mu1) ** (-n) * np.cos(np.pi * x) + 0.5 * (1 + p.dt * mu3) ** (-n) * np.cos(3 * np.pi * x)
    assert np.max(np.abs(U - (Un + exact))) < p.nt * (1 + p.dt * _lam(p.n - 1, p.n) ** 2) * 4.4e-16


def test_constant_state_is_steady():
    for op in ("biharmonic", "linear_ch"):
        U = stepper.theta_method(op, 2, 8, 5, 1e-4, np.full((8, 8), 0.37), eps=0.1, beta=0.3)
        assert np.max(np.abs(U - 0.37)) < 1e-14
    U = stepper.ch_implicit(2, 8, 5, 1e-5, np.full((8, 8), -0.2), eps=0.05)
    assert np.max(np.abs(U + 0.2)) < 1e-14
