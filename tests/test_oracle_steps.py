"""Pins of the oracle with nonuniform time steps (CPU only).

With steps dt_1..dt_{N_t} the time-step matrix of the scheme is no longer the
alpha-circulant of Section 2.1; the Section 1 discussion of direct
diagonalization with variable steps is the case the general path covers.

* Closed form: a cosine mode cos(k pi x) at the cell centres is an eigenvector
  of A, so under the theta-method it decays by exactly
  prod_n R_theta(dt_n mu_k) with R_theta(z) = (1 - (1-theta) z)/(1 + theta z).
* Brute force: the stepping equals a dense solve of the whole system
  (B (x) I + C (x) A) U = b written from its blocks, and for nonlinear CH a
  full Newton iteration on the dense all-at-once system with 1/dt_n in the
  time differences.
* Residual: the oracle's residual vanishes on the stepped solution and equals
  b at U = 0.
* The per-mode solve with (B + mu_k I) equals a sparse direct solve of the
  space-time system.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import allatonce as aao
from oracle import operators as ops
from oracle import stepper
from workloads import Problem, cell_centres, time_steps


def _graded(nt, dt=1e-5, q=1.3):
    return dt * q ** np.arange(nt)


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("op,eps,beta", [("biharmonic", 1.0, 0.0), ("linear_ch", 0.05, 0.5)])
def test_cosine_modes_decay_by_the_product_of_step_factors(theta, op, eps, beta):
    n, nt = 32, 12
    dts = _graded(nt, 2e-6, 1.3)
    x = cell_centres(n)
    h = 1.0 / n
    u0 = np.cos(np.pi * x) + 0.5 * np.cos(3 * np.pi * x)
    U = stepper.theta_method(op, 1, n, nt, 0.0, u0, theta=theta, eps=eps, beta=beta, dts=dts)
    expect = np.zeros_like(U)
    for k, c in ((1, 1.0), (3, 0.5)):
        lam = 2.0 / h ** 2 * (np.cos(k * np.pi / n) - 1.0)
        mu = lam * lam if op == "biharmonic" else beta ** 2 * lam + eps ** 2 * lam * lam
        z = dts * mu
        fac = np.cumprod((1 - (1 - theta) * z) / (1 + theta * z))
        expect += c * fac[:, None] * np.cos(k * np.pi * x)[None, :]
    assert np.max(np.abs(U - expect)) < 1e-13


@pytest.mark.parametrize("dim,n,nt", [(1, 6, 5), (2, 4, 4)])
@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("op", ["biharmonic", "linear_ch"])
def test_dense_system_with_steps_equals_stepping(dim, n, nt, theta, op):
    rng = np.random.default_rng(17)
    dts = _graded(nt, 1e-4, 1.5)
    u0 = rng.uniform(-1, 1, (n,) * dim)
    a = ops.operator_a(op, dim, n, 1.0 / n, eps=0.1, beta=0.4).toarray()
    ns = a.shape[0]
    # blocks written out: row n carries (u_n - u_{n-1})/dt_n + A(theta u_n + (1-theta) u_{n-1})
    K = np.zeros((nt * ns, nt * ns))
    for i in range(nt):
        K[i * ns:(i + 1) * ns, i * ns:(i + 1) * ns] = np.eye(ns) / dts[i] + theta * a
        if i:
            K[i * ns:(i + 1) * ns, (i - 1) * ns:i * ns] = -np.eye(ns) / dts[i] + (1 - theta) * a
    b = np.zeros(nt * ns)
    b[:ns] = u0.ravel() / dts[0] - (1 - theta) * a @ u0.ravel()
    dense = np.linalg.solve(K, b).reshape((nt,) + u0.shape)
    seq = stepper.theta_method(op, dim, n, nt, 0.0, u0, theta=theta, eps=0.1, beta=0.4, dts=dts)
    assert np.max(np.abs(dense - seq)) < 1e-12 * max(1.0, np.max(np.abs(seq)))
    kk = aao.allatonce_matrix_steps(ops.operator_a(op, dim, n, 1.0 / n, eps=0.1, beta=0.4), dts, theta).toarray()
    assert np.allclose(kk, K, rtol=0, atol=1e-9 * np.max(np.abs(K)))


@pytest.mark.parametrize("dim,n,nt", [(1, 8, 6), (2, 4, 4)])
def test_dense_newton_ch_with_steps_equals_stepping(dim, n, nt):
    rng = np.random.default_rng(23)
    dts = _graded(nt, 1e-4, 1.4)
    eps = 0.1
    u0 = rng.uniform(-0.8, 0.8, (n,) * dim)
    lap = ops.laplacian(dim, n, 1.0 / n).toarray()
    ns = lap.shape[0]
    B = (np.eye(nt) - np.eye(nt, k=-1)) / dts[:, None]
    K1 = np.kron(B, np.eye(ns))
    L = np.kron(np.eye(nt), lap)
    L2 = np.kron(np.eye(nt), lap @ lap)
    b = np.zeros(nt * ns)
    b[:ns] = u0.ravel() / dts[0]
    U = np.tile(u0.ravel(), nt)
    for _ in range(50):
        G = K1 @ U - L @ U ** 3 + L @ U + eps ** 2 * (L2 @ U) - b
        J = K1 - L @ np.diag(3 * U ** 2) + L + eps ** 2 * L2
        dU = np.linalg.solve(J, G)
        U -= dU
        if np.max(np.abs(dU)) < 1e-15:
            break
    seq = stepper.ch_implicit(dim, n, nt, 0.0, u0, eps, dts=dts)
    assert np.max(np.abs(U.reshape(seq.shape) - seq)) < 1e-12


@pytest.mark.parametrize("op", ["linear_ch", "ch"])
def test_residual_with_steps(op):
    p = Problem(op=op, dim=2, n=8, nt=6, dt=1e-5, eps=0.08, beta=0.4, q=1.4)
    dts = time_steps(p)
    rng = np.random.default_rng(4)
    u0 = rng.uniform(-0.3, 0.3, p.slice_shape)
    U = stepper.sequential(p, u0, dts)
    r = aao.residual_steps(p, U, u0, dts)
    scale = np.max(np.abs(U)) / np.min(dts)
    assert np.max(np.abs(r)) < 1e-11 * scale
    if op == "linear_ch":
        r0 = aao.residual_steps(p, np.zeros(p.shape), u0, dts)
        a = ops.operator_a(op, 2, p.n, p.h, eps=p.eps, beta=p.beta)
        assert np.allclose(r0[0].ravel(), u0.ravel() / dts[0], rtol=1e-15, atol=0)  # theta = 1: b_1 = u0 / dt_1
        assert np.all(r0[1:] == 0.0)
        assert a.shape[0] == p.ns


@pytest.mark.parametrize("op,c_bar,theta", [("linear_ch", 0.0, 1.0), ("biharmonic", 0.0, 1.0), ("ch", 0.37, 1.0),
                                            ("linear_ch", 0.0, 0.5), ("biharmonic", 0.0, 0.5)])
def test_modal_solve_with_steps_equals_direct_solve(op, c_bar, theta):
    p = Problem(op=op, dim=2, n=6, nt=5, dt=1e-5, eps=0.07, beta=0.4, q=1.6, theta=theta)
    dts = time_steps(p)
    rng = np.random.default_rng(6)
    r = rng.standard_normal(p.shape)
    if op == "ch":
        lap = ops.laplacian(2, p.n, p.h)
        a = ((1.0 - c_bar) * lap + p.eps ** 2 * (lap @ lap)).tocsr()
    else:
        a = ops.operator_a(op, 2, p.n, p.h, eps=p.eps, beta=p.beta)
    direct = spla.spsolve(aao.allatonce_matrix_steps(a, dts, theta).tocsc(), r.reshape(-1)).reshape(r.shape)
    modal = aao.idct2(aao.time_solve_steps_modal(p, aao.dct2(r, 2), dts, c_bar), 2)
    assert np.max(np.abs(modal - direct)) < 1e-11 * np.max(np.abs(direct))


def test_uniform_steps_reduce_to_the_circulant_blocks():
    dts = np.full(7, 3e-5)
    b, c = aao.step_blocks(dts, 0.5)
    c1, c2 = aao.circulant_blocks(7, 3e-5, 0.5, 0.0)
    assert np.allclose(b, c1, rtol=1e-15, atol=0) and np.array_equal(c, c2)
