"""Pins of the oracle's checkers and invariants (CPU only).

* The error norms every parity test uses (Section 5: the error in the discrete
  L^inf(0,T; L^2) norm, and its L^inf(L^inf) variant), on hand-built pairs
  whose answers are worked out by hand: an error at one level only (a mean
  over levels, or a per-level normalisation, would give another number) and
  a scaled copy (pins the normalisation by the reference's largest level).
* Mass: closed forms on the cell-centred grid (constants, a linear ramp,
  cosine modes), and conservation to roundoff by every sequential scheme
  (the Neumann problems conserve the integral of u, Section 1).
* Energy: the Ginzburg-Landau energy does not increase along the implicit and
  the Eyre CH steppers for dt << eps^2 (Section 4.1, the energy remarks after
  the fully discrete schemes; Eyre is unconditionally stable).
* The scalar averaged Jacobian on hand cases.
* The chord iteration's stop rule leaves dt ||F||_inf <= 1e-14 at every step.
"""
import numpy as np
import pytest

from oracle import allatonce as aao
from oracle import operators as ops
from oracle import stepper


# ------------------------------------------------------------- error norms
def _pair():
    # two levels of a 2 x 2 grid: level norms 2 (all ones) and 6 (all threes)
    ref = np.stack([np.ones((2, 2)), 3.0 * np.ones((2, 2))])
    return ref


def test_rel_err_error_at_one_level_only():
    ref = _pair()
    u = ref.copy()
    u[0, 0, 1] += 1.0          # ||e_1|| = 1 at the level with norm 2, nothing at level 2
    # max_n ||e_n|| / max_n ||ref_n|| = 1 / 6 (a per-level ratio would give 1/2,
    # a mean over levels 1/12)
    assert stepper.rel_err(u, ref) == pytest.approx(1.0 / 6.0, rel=1e-15)
    assert stepper.rel_err_inf(u, ref) == pytest.approx(1.0 / 3.0, rel=1e-15)


def test_rel_err_takes_the_max_over_levels():
    ref = _pair()
    u = ref.copy()
    u[0] += 0.5                # ||e_1|| = 0.5 * 2 = 1
    u[1, 1, 1] -= 2.0          # ||e_2|| = 2: the larger one counts
    assert stepper.rel_err(u, ref) == pytest.approx(2.0 / 6.0, rel=1e-15)
    assert stepper.rel_err_inf(u, ref) == pytest.approx(2.0 / 3.0, rel=1e-15)


def test_rel_err_scaled_copy():
    rng = np.random.default_rng(8)
    ref = rng.standard_normal((5, 7, 7))
    for s in (1e-3, 1e-11, 0.25):
        assert stepper.rel_err((1.0 + s) * ref, ref) == pytest.approx(s, rel=1e-4)
        assert stepper.rel_err_inf((1.0 - s) * ref, ref) == pytest.approx(s, rel=1e-4)
    assert stepper.rel_err(ref, ref) == 0.0 and stepper.rel_err_inf(ref, ref) == 0.0


# -------------------------------------------------------------------- mass
@pytest.mark.parametrize("dim,n", [(1, 10), (2, 6), (2, 16)])
def test_mass_closed_forms(dim, n):
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    shape = (n,) * dim
    assert ops.mass(np.full(shape, 0.7), h) == pytest.approx(0.7, rel=1e-14)
    # the midpoint rule integrates a linear function exactly: int_0^1 x dx = 1/2
    ramp = np.broadcast_to(x, shape)
    assert ops.mass(np.ascontiguousarray(ramp), h) == pytest.approx(0.5, rel=1e-14)
    # every non-constant cosine mode sums to zero over the cell centres
    for k in (1, 2, n - 1):
        c = np.broadcast_to(np.cos(k * np.pi * x), shape)
        assert abs(ops.mass(np.ascontiguousarray(c), h)) < 1e-15


def _level_masses(U, u0, h):
    return np.array([ops.mass(u0, h)] + [ops.mass(u, h) for u in U])


@pytest.mark.parametrize("op,theta", [("biharmonic", 1.0), ("biharmonic", 0.5), ("linear_ch", 1.0),
                                      ("linear_ch", 0.5)])
@pytest.mark.parametrize("dim", [1, 2])
def test_linear_steppers_conserve_mass(op, theta, dim):
    n, nt, dt = (32, 12, 1e-5) if dim == 1 else (16, 8, 1e-5)
    rng = np.random.default_rng(21 + dim)
    u0 = 0.3 + rng.uniform(-0.05, 0.05, (n,) * dim)
    U = stepper.theta_method(op, dim, n, nt, dt, u0, theta=theta, eps=0.05, beta=0.5)
    m = _level_masses(U, u0, 1.0 / n)
    assert np.max(np.abs(m - m[0])) <= 1e-13 * np.max(np.abs(m))


@pytest.mark.parametrize("scheme", ["implicit", "eyre"])
@pytest.mark.parametrize("dim", [1, 2])
def test_ch_steppers_conserve_mass_and_dissipate_energy(scheme, dim):
    n, nt, dt, eps = (64, 20, 1e-6, 0.02) if dim == 1 else (24, 10, 1e-6, 0.03)
    rng = np.random.default_rng(31 + dim)
    u0 = 0.1 + rng.uniform(-0.3, 0.3, (n,) * dim)
    run = stepper.ch_implicit if scheme == "implicit" else stepper.ch_eyre
    U = run(dim, n, nt, dt, u0, eps)
    h = 1.0 / n
    m = _level_masses(U, u0, h)
    assert np.max(np.abs(m - m[0])) <= 1e-13 * np.max(np.abs(m))
    e = np.array([ops.energy(u0, eps, h)] + [ops.energy(u, eps, h) for u in U])
    assert np.all(np.diff(e) <= 1e-13 * np.abs(e[1:])), np.diff(e)
    assert e[-1] < e[0]  # the random datum relaxes


def test_eyre_dissipates_energy_at_a_large_step():
    # Eyre's splitting is unconditionally energy stable: a step of eps^2 / 4,
    # 600 times the configurations' dt / eps^2, still lowers the energy.  (The
    # oracle's chord stop needs dt ||F||_inf to reach 1e-14, which bounds the
    # steps it accepts: at dt = 4 eps^2 the roundoff of F alone is ~2e-14.)
    n, nt, eps = 32, 6, 0.05
    dt = 0.25 * eps * eps
    u0 = np.random.default_rng(5).uniform(-0.5, 0.5, (n, n))
    U = stepper.ch_eyre(2, n, nt, dt, u0, eps)
    h = 1.0 / n
    e = np.array([ops.energy(u0, eps, h)] + [ops.energy(u, eps, h) for u in U])
    assert np.all(np.diff(e) <= 1e-13 * np.abs(e[1:])), np.diff(e)


# --------------------------------------------------- scalar averaged Jacobian
def test_mean_jacobian_hand_cases():
    U = np.array([[1.0, -1.0], [2.0, 0.0]])      # 3 (1 + 1 + 4 + 0) / 4
    assert aao.mean_jacobian(U) == 4.5
    assert aao.mean_jacobian(np.full((3, 4, 4), -0.5)) == pytest.approx(0.75, rel=1e-15)
    assert aao.mean_jacobian(np.zeros((2, 3))) == 0.0


# ---------------------------------------------------------- chord stop rule
@pytest.mark.parametrize("scheme", ["implicit", "eyre"])
def test_chord_steps_settle_the_step_equation(scheme):
    n, nt, dt, eps = 20, 5, 1e-6, 0.02
    u0 = np.random.default_rng(9).uniform(-0.1, 0.1, (n, n))
    run = stepper.ch_implicit if scheme == "implicit" else stepper.ch_eyre
    U, iters = run(2, n, nt, dt, u0, eps, return_iters=True)
    lap = ops.laplacian(2, n, 1.0 / n)
    prev = u0.reshape(-1)
    for k in range(nt):
        f = stepper.ch_residual(U[k].reshape(-1), prev, lap, dt, eps, scheme)
        assert dt * np.max(np.abs(f)) <= 1e-14
        prev = U[k].reshape(-1)
    assert all(1 <= i <= stepper.NEWTON_MAXIT for i in iters)


# ------------------------------------------ space-varying averaged Jacobian
def test_jacobian_field_hand_case():
    U = np.array([[[1.0, -2.0]], [[3.0, 0.0]]])   # two levels of a 1 x 2 grid
    assert np.array_equal(aao.jacobian_field(U), np.array([[3.0 * (1 + 9) / 2, 3.0 * (4 + 0) / 2]]))
    assert aao.jacobian_field(U).mean() == aao.mean_jacobian(U)


def test_field_jacobian_with_a_constant_field_is_the_scalar_preconditioner():
    from workloads import Problem
    p = Problem(op="ch", dim=2, n=6, nt=4, dt=1e-5, eps=0.1, alpha=0.02)
    a = aao.precond_matrix_field(p, np.full((6, 6), 0.37)).toarray()
    b = aao.precond_matrix(p, 0.37).toarray()
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_field_jacobian_is_the_exact_jacobian_for_a_time_constant_iterate():
    # When every level holds the same field w, the time average of J_s is J_s(w):
    # with alpha = 0 the approximate Jacobian G~' is then the exact derivative of
    # the residual map G (eq. jacobian1), checked by central differences.
    from workloads import Problem
    p = Problem(op="ch", dim=2, n=5, nt=3, dt=1e-4, eps=0.2, alpha=0.0)
    rng = np.random.default_rng(21)
    w = rng.uniform(-0.8, 0.8, p.slice_shape)
    U = np.broadcast_to(w, p.shape).copy()
    u0 = rng.uniform(-0.8, 0.8, p.slice_shape)
    m = aao.precond_matrix_field(p, aao.jacobian_field(U)).toarray()
    V = rng.standard_normal(p.shape)
    h = 1e-6
    # G = -residual (the residual is b - K(U))
    dG = (-aao.residual(p, U + h * V, u0) + aao.residual(p, U - h * V, u0)) / (2 * h)
    assert np.max(np.abs(m @ V.reshape(-1) - dG.reshape(-1))) <= 1e-6 * np.max(np.abs(dG))
