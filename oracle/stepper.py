"""Sequential fully discrete time stepping (test infrastructure, FP64).

These are the schemes whose solution the parallel-in-time iteration converges
to.  Each step is a direct spatial solve with LAPACK banded Cholesky
(``scipy.linalg.cholesky_banded`` / ``cho_solve_banded``); nonlinear steps
iterate on the frozen SPD matrix until both the increment (relative) and the
scaled step residual dt ||F||_inf are below 1e-14.  No fast
transform is used; ``ch_step_modal`` (single steps on grids too large to
factor) inverts the frozen matrix with the explicit dense cosine matrix.

Schemes
-------
theta_method   (u_n - u_{n-1})/dt + A (theta u_n + (1-theta) u_{n-1}) = 0
               (Section 2.1, eq. linear-theta1 with alpha = 0; A from
               operators.operator_a).  theta = 1 is backward Euler.
               Every scheme also takes nonuniform steps dt_n (the general
               time-step matrix of the Section 1 discussion of direct
               diagonalization with variable steps).
ch_implicit    (u_n - u_{n-1})/dt = Lap_h(u_n^3 - u_n) - eps^2 Lap_h^2 u_n
               (Section 4.1, eq. fully-dis_CH: the fully implicit scheme of
               PinT-I).
ch_eyre        (u_n - u_{n-1})/dt = Lap_h u_n^3 - Lap_h u_{n-1} - eps^2 Lap_h^2 u_n
               (Section 4.1, eq. fully-dis_CH_WR_Eyre with alpha = 0: Eyre's
               convex/concave splitting of PinT-II).

All return the space-time array [N_t][...] holding u_1..u_{N_t}; u_0 is the
given datum and is not part of the output.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import operators as ops

NEWTON_TOL = 1e-14
NEWTON_MAXIT = 200


class _BandedSPD:
    """LAPACK banded Cholesky factor of a symmetric positive definite sparse matrix."""

    def __init__(self, m: sp.spmatrix):
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        ab, self.b = ops.sym_band_upper(m)
        self.cb = sla.cholesky_banded(ab, lower=False)

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        return sla.cho_solve_banded((self.cb, False), rhs)


def _steps(nt: int, dt: float, dts):
    """The step of each level: dts[n-1] when given (nonuniform steps), else dt."""
    if dts is None:
        return [dt] * nt
    dts = np.asarray(dts, dtype=np.float64)
    if dts.shape != (nt,) or not np.all(dts > 0):
        raise ValueError("dts must hold nt positive steps")
    return [float(x) for x in dts]


def theta_method(op: str, dim: int, n: int, nt: int, dt: float, u0: np.ndarray,
                 theta: float = 1.0, eps: float = 1.0, beta: float = 0.0, dts=None) -> np.ndarray:
    """Sequential linear theta-method (Section 2.1, eq. linear-theta1, alpha=0).

    Solves (I + theta dt_n A) u_n = (I - (1-theta) dt_n A) u_{n-1}, n = 1..nt,
    with dt_n = dt, or dts[n-1] for nonuniform steps.  The matrix is SPD
    whenever 1 + theta dt_n mu_min > 0 (mu_min the smallest eigenvalue of A,
    negative for the spinodal linearized CH operator); a non-SPD matrix makes
    the Cholesky factorization raise.
    """
    h = 1.0 / n
    a = ops.operator_a(op, dim, n, h, eps=eps, beta=beta)
    eye = sp.identity(a.shape[0], format="csr")
    facs = {}
    u = np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    out = np.empty((nt, u.size))
    for k, dk in enumerate(_steps(nt, dt, dts)):
        if dk not in facs:  # one factorization per distinct step
            facs[dk] = (_BandedSPD(eye + theta * dk * a), (eye - (1.0 - theta) * dk * a).tocsr())
        lhs, rhs_op = facs[dk]
        u = lhs.solve(rhs_op @ u)
        out[k] = u
    return out.reshape((nt,) + (n,) * dim)


def ch_residual(u: np.ndarray, u_prev: np.ndarray, lap: sp.spmatrix, dt: float, eps: float,
                scheme: str = "implicit") -> np.ndarray:
    """Per-step residual F(u) of the nonlinear CH schemes (flattened arrays).

    implicit: F(u) = (u - u_prev)/dt - Lap_h(u^3 - u) + eps^2 Lap_h^2 u   (eq. fully-dis_CH)
    eyre    : F(u) = (u - u_prev)/dt - Lap_h u^3 + Lap_h u_prev + eps^2 Lap_h^2 u
    """
    lu = lap @ u
    if scheme == "implicit":
        return (u - u_prev) / dt - lap @ (u * u * u - u) + eps * eps * (lap @ lu)
    if scheme == "eyre":
        return (u - u_prev) / dt - lap @ (u * u * u) + lap @ u_prev + eps * eps * (lap @ lu)
    raise ValueError(scheme)


def _chord(u: np.ndarray, solve, resid, dt: float):
    """Chord iteration u <- u - J0^{-1} F(u) for one nonlinear step.  Stops when
    the last increment satisfies ||du||_inf <= 1e-14 max(1, ||u||_inf) and the
    scaled residual of the new iterate satisfies dt ||F(u)||_inf <= 1e-14, so
    that both the iterate and the step equation are settled to roundoff.
    Returns (u, number of increments), or (u, None) at the iteration cap."""
    small_step = False
    for it in range(NEWTON_MAXIT + 1):
        f = resid(u)
        if small_step and dt * np.max(np.abs(f)) <= NEWTON_TOL:
            return u, it
        if it == NEWTON_MAXIT:
            break
        du = solve(f)
        u = u - du
        small_step = np.max(np.abs(du)) <= NEWTON_TOL * max(1.0, np.max(np.abs(u)))
    return u, None


def _ch_steps(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float, scheme: str,
              return_iters: bool = False, dts=None):
    h = 1.0 / n
    lap = ops.laplacian(dim, n, h)
    lap2 = (lap @ lap).tocsr()
    eye = sp.identity(lap.shape[0], format="csr")
    facs = {}

    def frozen(dk):
        # Frozen Jacobian: the derivative of F at u = 0.  It is SPD for the
        # implicit scheme iff 1/dt > 1/(4 eps^2) (the minimum of lam + eps^2
        # lam^2 over lam <= 0 is -1/(4 eps^2)); for Eyre it is always SPD.
        if dk not in facs:
            if scheme == "implicit":
                j0 = eye / dk + lap + eps * eps * lap2
            else:
                j0 = eye / dk + eps * eps * lap2
            facs[dk] = _BandedSPD(j0)
        return facs[dk]

    u = np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    out = np.empty((nt, u.size))
    iters = []
    for k, dk in enumerate(_steps(nt, dt, dts)):
        u_prev = u.copy()
        fac = frozen(dk)
        u, it = _chord(u, lambda f: fac.solve(f), lambda v: ch_residual(v, u_prev, lap, dk, eps, scheme), dk)
        if it is None:
            raise RuntimeError(f"CH step {k + 1}: chord iteration did not converge")
        iters.append(it)
        out[k] = u
    res = out.reshape((nt,) + (n,) * dim)
    return (res, iters) if return_iters else res


def ch_implicit(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float,
                return_iters: bool = False, dts=None):
    """Fully implicit backward-Euler CH (Section 4.1, eq. fully-dis_CH), each step
    solved by chord iterations on the frozen SPD matrix I/dt + Lap_h + eps^2 Lap_h^2
    to ||du||_inf <= 1e-14 max(1, ||u||_inf) and dt ||F(u)||_inf <= 1e-14.
    dts: nonuniform steps (dt_n = dts[n-1]) instead of dt."""
    return _ch_steps(dim, n, nt, dt, u0, eps, "implicit", return_iters, dts)


def ch_eyre(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float,
            return_iters: bool = False, dts=None):
    """Eyre's convex/concave split CH (Section 4.1, eq. fully-dis_CH_WR_Eyre with
    alpha = 0): u^3 implicit, the -u part explicit."""
    return _ch_steps(dim, n, nt, dt, u0, eps, "eyre", return_iters, dts)


def ch_step_modal(u_prev: np.ndarray, dt: float, eps: float, scheme: str = "implicit") -> np.ndarray:
    """One CH step (eq. fully-dis_CH, or the Eyre scheme) from the 2D or 1D
    level u_prev, for grids where a banded factorization is too large.

    Same chord iteration as ``ch_implicit`` / ``ch_eyre`` (frozen matrix
    J0 = I/dt + Lap_h + eps^2 Lap_h^2, resp. I/dt + eps^2 Lap_h^2, same 1e-14
    stop), but J0 is inverted in the explicit orthonormal cosine basis:
    J0 = Q^T diag(j) Q with Q = allatonce.dct2_matrix(N) applied along each
    axis and j the eigenvalues from the Laplacian spectrum.  Pinned against the
    banded-Cholesky steppers on small grids.
    """
    from .allatonce import dct2_matrix
    u_prev = np.asarray(u_prev, dtype=np.float64)
    dim = u_prev.ndim
    n = u_prev.shape[-1]
    h = 1.0 / n
    q = dct2_matrix(n)
    lam1 = ops.spectrum_1d(n, h)
    lam = lam1 if dim == 1 else lam1[:, None] + lam1[None, :]
    jdiag = 1.0 / dt + eps * eps * lam * lam + (lam if scheme == "implicit" else 0.0)

    def fwd(x):
        return q @ x if dim == 1 else q @ x @ q.T

    def inv(x):
        return q.T @ x if dim == 1 else q.T @ x @ q

    lap = ops.laplacian(dim, n, h)
    up = u_prev.reshape(-1)
    u, it = _chord(up.copy(), lambda f: inv(fwd(f.reshape(u_prev.shape)) / jdiag).reshape(-1),
                   lambda v: ch_residual(v, up, lap, dt, eps, scheme), dt)
    if it is None:
        raise RuntimeError("modal CH step: chord iteration did not converge")
    return u.reshape(u_prev.shape)


def sequential(problem, u0: np.ndarray, dts=None) -> np.ndarray:
    """Solve a ``workloads.Problem`` by the matching sequential scheme.  A
    problem with nonuniform steps (growth ratio q != 1) needs its steps dts."""
    p = problem
    if getattr(p, "q", 1.0) != 1.0 and dts is None:
        raise ValueError("a problem with nonuniform steps needs dts")
    if p.op in ("biharmonic", "linear_ch"):
        return theta_method(p.op, p.dim, p.n, p.nt, p.dt, u0, theta=p.theta, eps=p.eps, beta=p.beta, dts=dts)
    if p.op == "ch":
        return ch_implicit(p.dim, p.n, p.nt, p.dt, u0, p.eps, dts=dts)
    if p.op == "ch_eyre":
        return ch_eyre(p.dim, p.n, p.nt, p.dt, u0, p.eps, dts=dts)
    raise ValueError(p.op)


def rel_err(u: np.ndarray, ref: np.ndarray) -> float:
    """Discrete L^inf(0,T; L^2) relative error max_n ||u_n - ref_n||_2 / max_n ||ref_n||_2
    (the paper's error norm, Section 5)."""
    nt = ref.shape[0]
    d = np.sqrt(np.sum((u - ref).reshape(nt, -1) ** 2, axis=1))
    r = np.sqrt(np.sum(ref.reshape(nt, -1) ** 2, axis=1))
    return float(np.max(d) / np.max(r))


def rel_err_inf(u: np.ndarray, ref: np.ndarray) -> float:
    """L^inf(0,T; L^inf) relative variant."""
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))
