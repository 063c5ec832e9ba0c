"""Brute-force pins on tiny grids (CPU only).

* The sequential stepping equals a dense solve of the whole all-at-once system
  with alpha = 0 (Section 2.1, eqs. all-at-once1 and ciculantmat; the
  alpha = 0 system is the sequential scheme gathered over all levels).
* For nonlinear CH, full Newton on the dense all-at-once system built from
  the Kronecker blocks of eq. nonlinear_G equals sequential chord stepping.
* The per-step CH residual is checked term by term against a closed form: for
  a single cosine mode u = A cos(k pi x), u^3 = A^3 (3 cos(k pi x) +
  cos(3k pi x))/4 pointwise, and every cosine cos(m pi x) is an eigenvector of
  the cell-centred Laplacian.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import allatonce as aao
from oracle import operators as ops
from oracle import stepper
from workloads import Problem, cell_centres


@pytest.mark.parametrize("dim,n,nt", [(1, 6, 5), (2, 4, 4)])
@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("op", ["biharmonic", "linear_ch"])
def test_dense_allatonce_equals_stepping(dim, n, nt, theta, op):
    rng = np.random.default_rng(11)
    dt = 1e-4
    u0 = rng.uniform(-1, 1, (n,) * dim)
    a = ops.operator_a(op, dim, n, 1.0 / n, eps=0.1, beta=0.4)
    # dense Kronecker system written from the block matrices directly
    c1 = (np.eye(nt) - np.eye(nt, k=-1)) / dt
    c2 = theta * np.eye(nt) + (1 - theta) * np.eye(nt, k=-1)
    ad = a.toarray()
    k = np.kron(c1, np.eye(ad.shape[0])) + np.kron(c2, ad)
    b = np.zeros(nt * ad.shape[0])
    b[: ad.shape[0]] = u0.ravel() / dt - (1 - theta) * ad @ u0.ravel()
    dense = np.linalg.solve(k, b).reshape((nt,) + u0.shape)
    seq = stepper.theta_method(op, dim, n, nt, dt, u0, theta=theta, eps=0.1, beta=0.4)
    assert np.max(np.abs(dense - seq)) < 1e-12 * max(1.0, np.max(np.abs(seq)))
    # and the oracle's own Kronecker assembly gives the same matrix
    kk = aao.allatonce_matrix(a, nt, dt, theta, 0.0).toarray()
    assert np.allclose(kk, k, rtol=0, atol=1e-9 * np.max(np.abs(k)))


def _dense_newton_ch(dim, n, nt, dt, eps, u0, scheme):
    h = 1.0 / n
    lap = ops.laplacian(dim, n, h).toarray()
    ns = lap.shape[0]
    c1 = (np.eye(nt) - np.eye(nt, k=-1)) / dt
    I = np.eye(ns)
    It = np.eye(nt)
    K1 = np.kron(c1, I)
    L = np.kron(It, lap)
    L2 = np.kron(It, lap @ lap)
    Sub = np.kron(np.eye(nt, k=-1), lap)   # C3^(0) (x) Lap_h
    b = np.zeros(nt * ns)
    b[:ns] = u0.ravel() / dt
    if scheme == "eyre":
        b[:ns] -= lap @ u0.ravel()

    def G(U):
        g = K1 @ U - L @ U ** 3 + eps ** 2 * (L2 @ U) - b
        return g + (Sub @ U if scheme == "eyre" else L @ U)

    def J(U):
        j = K1 - L @ np.diag(3 * U ** 2) + eps ** 2 * L2
        return j + (Sub if scheme == "eyre" else L)

    U = np.tile(u0.ravel(), nt)
    for _ in range(50):
        dU = np.linalg.solve(J(U), G(U))
        U -= dU
        if np.max(np.abs(dU)) < 1e-15:
            break
    return U.reshape((nt,) + u0.shape), np.max(np.abs(G(U)))


@pytest.mark.parametrize("scheme", ["implicit", "eyre"])
@pytest.mark.parametrize("dim,n,nt", [(1, 8, 6), (2, 4, 4)])
def test_dense_newton_ch_equals_stepping(scheme, dim, n, nt):
    rng = np.random.default_rng(5)
    dt, eps = 1e-4, 0.1
    u0 = rng.uniform(-0.8, 0.8, (n,) * dim)
    dense, gres = _dense_newton_ch(dim, n, nt, dt, eps, u0, scheme)
    assert gres < 1e-6  # G carries 1/dt and 1/h^4 scales
    if scheme == "implicit":
        seq = stepper.ch_implicit(dim, n, nt, dt, u0, eps)
    else:
        seq = stepper.ch_eyre(dim, n, nt, dt, u0, eps)
    assert np.max(np.abs(dense - seq)) < 1e-12


def test_ch_residual_single_mode_closed_form():
    n, dt, eps = 32, 1e-4, 0.07
    h = 1.0 / n
    x = cell_centres(n)
    lap = ops.laplacian(1, n, h)

    def lam(m):
        return 2.0 / h ** 2 * (np.cos(m * np.pi / n) - 1.0)

    k, amp, bprev = 2, 0.6, 0.3
    u = amp * np.cos(k * np.pi * x)
    u_prev = bprev * np.cos(k * np.pi * x)
    # Lap_h u^3 = amp^3 (3 lam_k cos(k pi x) + lam_3k cos(3k pi x)) / 4
    lap_u3 = amp ** 3 * (3 * lam(k) * np.cos(k * np.pi * x) + lam(3 * k) * np.cos(3 * k * np.pi * x)) / 4
    closed_impl = ((amp - bprev) / dt * np.cos(k * np.pi * x) - lap_u3
                   + lam(k) * u + eps ** 2 * lam(k) ** 2 * u)
    got = stepper.ch_residual(u, u_prev, lap, dt, eps, "implicit")
    assert np.max(np.abs(got - closed_impl)) < 1e-9 * np.max(np.abs(closed_impl))
    closed_eyre = ((amp - bprev) / dt * np.cos(k * np.pi * x) - lap_u3
                   + lam(k) * u_prev + eps ** 2 * lam(k) ** 2 * u)
    got = stepper.ch_residual(u, u_prev, lap, dt, eps, "eyre")
    assert np.max(np.abs(got - closed_eyre)) < 1e-9 * np.max(np.abs(closed_eyre))


def test_ch_steps_satisfy_pinned_residual():
    rng = np.random.default_rng(8)
    n, nt, dt, eps = 16, 6, 1e-5, 0.05
    u0 = rng.uniform(-0.5, 0.5, (n, n))
    U = stepper.ch_implicit(2, n, nt, dt, u0, eps)
    lap = ops.laplacian(2, n, 1.0 / n)
    prev = u0.ravel()
    for k in range(nt):
        F = stepper.ch_residual(U[k].ravel(), prev, lap, dt, eps)
        assert np.max(np.abs(F)) * dt < 1e-12
        prev = U[k].ravel()


def test_ch_small_amplitude_is_linearized_ch():
    # f'(0) = -1: CH linearized at u = 0 is u_t = -Lap u - eps^2 Lap^2 u,
    # i.e. the linearized CH equation with beta^2 = 1 (Section 3)
    rng = np.random.default_rng(9)
    n, nt, dt, eps, amp = 16, 8, 1e-5, 0.05, 1e-6
    u0 = amp * rng.uniform(-1, 1, (n, n))
    ch = stepper.ch_implicit(2, n, nt, dt, u0, eps)
    lin = stepper.theta_method("linear_ch", 2, n, nt, dt, u0, eps=eps, beta=1.0)
    assert np.max(np.abs(ch - lin)) < 1e-10 * amp


def test_residual_level_form_matches_kronecker():
    rng = np.random.default_rng(2)
    p = Problem(op="linear_ch", dim=2, n=6, nt=5, dt=1e-4, theta=0.5, eps=0.1, beta=0.3)
    u0 = rng.uniform(-1, 1, (6, 6))
    U = rng.uniform(-1, 1, p.shape)
    r = aao.residual_linear(p, U, u0)
    rl = aao.residual_linear_levels(p, U, u0, range(1, p.nt + 1))
    assert np.max(np.abs(r - rl)) < 1e-9 * np.max(np.abs(r))
    # the sequential solution has zero residual
    S = stepper.sequential(p, u0)
    r0 = aao.residual_linear(p, S, u0)
    assert np.max(np.abs(r0)) * p.dt < 1e-11


@pytest.mark.parametrize("scheme", ["implicit", "eyre"])
@pytest.mark.parametrize("dim,n", [(2, 16), (1, 32)])
def test_modal_ch_step_equals_banded_step(scheme, dim, n):
    rng = np.random.default_rng(31)
    dt, eps = 1e-5, 0.03
    u0 = rng.uniform(-0.6, 0.6, (n,) * dim)
    ref = (stepper.ch_implicit if scheme == "implicit" else stepper.ch_eyre)(dim, n, 1, dt, u0, eps)[0]
    got = stepper.ch_step_modal(u0, dt, eps, scheme)
    assert np.max(np.abs(got - ref)) < 1e-13
