"""Sequential fully discrete time stepping (test infrastructure, FP64).

These are the schemes whose solution the parallel-in-time iteration converges
to.  Each step is a direct spatial solve with LAPACK banded Cholesky
(``scipy.linalg.cholesky_banded`` / ``cho_solve_banded``); nonlinear steps
iterate on the frozen SPD matrix to a 1e-14 relative increment.  No fast
transform is used; ``ch_step_modal`` (single steps on grids too large to
factor) inverts the frozen matrix with the explicit dense cosine matrix.

Schemes
-------
theta_method   (u_n - u_{n-1})/dt + A (theta u_n + (1-theta) u_{n-1}) = 0
               (Section 2.1, eq. linear-theta1 with alpha = 0; A from
               operators.operator_a).  theta = 1 is backward Euler.
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


def theta_method(op: str, dim: int, n: int, nt: int, dt: float, u0: np.ndarray,
                 theta: float = 1.0, eps: float = 1.0, beta: float = 0.0) -> np.ndarray:
    """Sequential linear theta-method (Section 2.1, eq. linear-theta1, alpha=0).

    Solves (I + theta dt A) u_n = (I - (1-theta) dt A) u_{n-1}, n = 1..nt.  The
    matrix is SPD whenever 1 + theta dt mu_min > 0 (mu_min the smallest
    eigenvalue of A, negative for the spinodal linearized CH operator); a
    non-SPD matrix makes the Cholesky factorization raise.
    """
    h = 1.0 / n
    a = ops.operator_a(op, dim, n, h, eps=eps, beta=beta)
    eye = sp.identity(a.shape[0], format="csr")
    lhs = _BandedSPD(eye + theta * dt * a)
    rhs_op = (eye - (1.0 - theta) * dt * a).tocsr()
    u = np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    out = np.empty((nt, u.size))
    for k in range(nt):
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


def _ch_steps(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float, scheme: str,
              return_iters: bool = False):
    h = 1.0 / n
    lap = ops.laplacian(dim, n, h)
    lap2 = (lap @ lap).tocsr()
    eye = sp.identity(lap.shape[0], format="csr")
    # Frozen Jacobian: the derivative of F at u = 0.  It is SPD for the
    # implicit scheme iff 1/dt > 1/(4 eps^2) (the minimum of lam + eps^2 lam^2
    # over lam <= 0 is -1/(4 eps^2)); for Eyre it is always SPD.
    if scheme == "implicit":
        j0 = eye / dt + lap + eps * eps * lap2
    else:
        j0 = eye / dt + eps * eps * lap2
    fac = _BandedSPD(j0)
    u = np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    out = np.empty((nt, u.size))
    iters = []
    for k in range(nt):
        u_prev = u.copy()
        for it in range(NEWTON_MAXIT):
            du = fac.solve(ch_residual(u, u_prev, lap, dt, eps, scheme))
            u = u - du
            if np.max(np.abs(du)) <= NEWTON_TOL * max(1.0, np.max(np.abs(u))):
                break
        else:
            raise RuntimeError(f"CH step {k + 1}: chord iteration did not converge")
        iters.append(it + 1)
        out[k] = u
    res = out.reshape((nt,) + (n,) * dim)
    return (res, iters) if return_iters else res


def ch_implicit(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float,
                return_iters: bool = False):
    """Fully implicit backward-Euler CH (Section 4.1, eq. fully-dis_CH), each step
    solved by chord iterations on the frozen SPD matrix I/dt + Lap_h + eps^2 Lap_h^2
    to ||du||_inf <= 1e-14 max(1, ||u||_inf)."""
    return _ch_steps(dim, n, nt, dt, u0, eps, "implicit", return_iters)


def ch_eyre(dim: int, n: int, nt: int, dt: float, u0: np.ndarray, eps: float,
            return_iters: bool = False):
    """Eyre's convex/concave split CH (Section 4.1, eq. fully-dis_CH_WR_Eyre with
    alpha = 0): u^3 implicit, the -u part explicit."""
    return _ch_steps(dim, n, nt, dt, u0, eps, "eyre", return_iters)


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
    u = up.copy()
    for _ in range(NEWTON_MAXIT):
        f = ch_residual(u, up, lap, dt, eps, scheme).reshape(u_prev.shape)
        du = inv(fwd(f) / jdiag).reshape(-1)
        u = u - du
        if np.max(np.abs(du)) <= NEWTON_TOL * max(1.0, np.max(np.abs(u))):
            return u.reshape(u_prev.shape)
    raise RuntimeError("modal CH step: chord iteration did not converge")


def sequential(problem, u0: np.ndarray) -> np.ndarray:
    """Solve a ``workloads.Problem`` by the matching sequential scheme."""
    p = problem
    if p.op in ("biharmonic", "linear_ch"):
        return theta_method(p.op, p.dim, p.n, p.nt, p.dt, u0, theta=p.theta, eps=p.eps, beta=p.beta)
    if p.op == "ch":
        return ch_implicit(p.dim, p.n, p.nt, p.dt, u0, p.eps)
    if p.op == "ch_eyre":
        return ch_eyre(p.dim, p.n, p.nt, p.dt, u0, p.eps)
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
