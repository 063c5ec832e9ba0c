"""All-at-once (space-time) formulation, written out from its definitions
(test infrastructure, FP64).

Everything here is a plain matrix definition or a direct solve; nothing is
diagonalized by an FFT.  The functions serve as stage oracles (residual,
preconditioner application, spatial cosine transform) and as the reference
implementation of the outer iteration.

Readings of the paper fixed here
--------------------------------
* The residual the outer loop drives to zero is the alpha = 0 all-at-once
  residual r = b_0 - K(U), where K is the sequential scheme gathered over all
  time levels (eq. all-at-once1 / eq. all-at-once_CH with alpha = 0).  One
  quasi-Newton step per waveform-relaxation sweep, written in correction form
  U <- U + P_alpha^{-1} r(U), is the same iterate as the paper's
  P_alpha U^k = b^{k-1} (the alpha u_{N_t}^{k-1} terms of b^{k-1} cancel
  against the alpha-corner of P_alpha applied to U^{k-1}).
* The time-averaged Jacobian of PinT-I (eq. approx_jacobian) is taken as a
  scalar c_bar I with c_bar the space-time mean of 3 u^2, so that the Step-(2)
  operator stays diagonal in the cosine basis.  This changes the
  preconditioner only, not the fixed point.
* J_s(u) is read as diag(3 u^2), the derivative of u^3 (the printed
  diag((3u)^2) is taken as a typesetting slip).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as ops


# ---------------------------------------------------------------- time blocks
def circulant_blocks(nt: int, dt: float, theta: float, alpha: float):
    """Strang-type alpha-circulant matrices C1, C2 (Section 2.1, eq. ciculantmat).

    C1 = (1/dt) [1 on the diagonal, -1 on the subdiagonal, -alpha in the top-right corner]
    C2 = [theta on the diagonal, 1-theta on the subdiagonal, (1-theta) alpha top-right]
    With alpha = 0 they are the sequential theta-method in time.
    """
    c1 = np.eye(nt) - np.eye(nt, k=-1)
    c1[0, nt - 1] = -alpha
    c1 /= dt
    c2 = theta * np.eye(nt) + (1.0 - theta) * np.eye(nt, k=-1)
    c2[0, nt - 1] = (1.0 - theta) * alpha
    return c1, c2


def step_blocks(dts, theta: float = 1.0):
    """Time-step matrices of the theta-method with nonuniform steps dt_n
    (alpha = 0): B = diag(1/dt_n) (I - S) and C = theta I + (1 - theta) S,
    S the down-shift, so that the scheme over all levels reads
    (B (x) I + C (x) A) U = b.  With equal steps B = C1^(0) and C = C2^(0)
    of eq. ciculantmat.  Unlike C1^(alpha), B is not alpha-circulant; it is
    diagonalized directly (Section 1: direct diagonalization with variable
    steps)."""
    dts = np.asarray(dts, dtype=np.float64)
    nt = dts.size
    b = (np.eye(nt) - np.eye(nt, k=-1)) / dts[:, None]
    c = theta * np.eye(nt) + (1.0 - theta) * np.eye(nt, k=-1)
    return b, c


def c3_block(nt: int, alpha: float):
    """C3 = C2 with theta = 0 (Section 4.1, after eq. all-at-once_CH_Eyre)."""
    _, c3 = circulant_blocks(nt, 1.0, 0.0, alpha)
    return c3


def allatonce_matrix(a: sp.spmatrix, nt: int, dt: float, theta: float, alpha: float) -> sp.csr_matrix:
    """C1^(alpha) (x) I + C2^(alpha) (x) A (Section 2.1, eq. all-at-once1)."""
    c1, c2 = circulant_blocks(nt, dt, theta, alpha)
    eye = sp.identity(a.shape[0], format="csr")
    return (sp.kron(sp.csr_matrix(c1), eye) + sp.kron(sp.csr_matrix(c2), a)).tocsr()


def rhs_linear(u0: np.ndarray, a: sp.spmatrix, nt: int, dt: float, theta: float,
               alpha: float = 0.0, u_nt_prev=None) -> np.ndarray:
    """b^{k-1}: first block (I/dt - (1-theta) A)(u0 - alpha u_{N_t}^{k-1}), the
    other blocks zero (Section 2.1, after eq. ciculantmat; A symmetric so the
    row-vector form printed there is the same vector)."""
    ns = a.shape[0]
    w = np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    if alpha != 0.0:
        w = w - alpha * np.asarray(u_nt_prev).reshape(-1)
    b = np.zeros(nt * ns)
    b[:ns] = w / dt - (1.0 - theta) * (a @ w)
    return b


def allatonce_matrix_steps(a: sp.spmatrix, dts, theta: float) -> sp.csr_matrix:
    """B (x) I + C (x) A for nonuniform steps (``step_blocks``)."""
    b, c = step_blocks(dts, theta)
    eye = sp.identity(a.shape[0], format="csr")
    return (sp.kron(sp.csr_matrix(b), eye) + sp.kron(sp.csr_matrix(c), a)).tocsr()


def rhs_steps(u0: np.ndarray, a: sp.spmatrix, dts, theta: float) -> np.ndarray:
    """First block u0/dt_1 - (1-theta) A u0, the others zero."""
    dts = np.asarray(dts, dtype=np.float64)
    ns = a.shape[0]
    w = np.asarray(u0, dtype=np.float64).reshape(-1)
    b = np.zeros(dts.size * ns)
    b[:ns] = w / dts[0] - (1.0 - theta) * (a @ w)
    return b


# ------------------------------------------------------------------ residuals
def residual_linear(p, U: np.ndarray, u0: np.ndarray) -> np.ndarray:
    """True alpha = 0 residual r = b_0 - (C1^(0) (x) I + C2^(0) (x) A) U of the
    linear theta-method (eq. all-at-once1 with alpha = 0), as a Kronecker
    matrix-vector product.  U is [N_t][...]; returns the same shape."""
    a = ops.operator_a(p.op, p.dim, p.n, p.h, eps=p.eps, beta=p.beta)
    k = allatonce_matrix(a, p.nt, p.dt, p.theta, 0.0)
    b = rhs_linear(u0, a, p.nt, p.dt, p.theta)
    return (b - k @ U.reshape(-1)).reshape(U.shape)


def residual_steps(p, U: np.ndarray, u0: np.ndarray, dts) -> np.ndarray:
    """True residual r = b - K(U) of the sequential scheme with nonuniform
    steps (linear: (B (x) I + C (x) A); CH: eq. nonlinear_G with 1/dt_n in
    the time difference of level n), all levels."""
    dts = np.asarray(dts, dtype=np.float64)
    if p.op in ("biharmonic", "linear_ch"):
        a = ops.operator_a(p.op, p.dim, p.n, p.h, eps=p.eps, beta=p.beta)
        k = allatonce_matrix_steps(a, dts, p.theta)
        return (rhs_steps(u0, a, dts, p.theta) - k @ U.reshape(-1)).reshape(U.shape)
    lap = ops.laplacian(p.dim, p.n, p.h)
    e2 = p.eps * p.eps
    out = []
    for n in range(1, p.nt + 1):
        un = U[n - 1].reshape(-1)
        um = (u0 if n == 1 else U[n - 2]).reshape(-1)
        if p.op == "ch":
            g = (un - um) / dts[n - 1] - lap @ (un ** 3) + lap @ un + e2 * (lap @ (lap @ un))
        else:
            raise ValueError(f"nonuniform steps: no residual for {p.op}")
        out.append(-g)
    return np.array(out).reshape(U.shape)


def residual_linear_levels(p, U: np.ndarray, u0: np.ndarray, levels) -> np.ndarray:
    """The same residual evaluated level by level, for the given time levels
    only (1-based n as in the paper):
    r_n = -[(u_n - u_{n-1})/dt + A(theta u_n + (1-theta) u_{n-1})]."""
    a = ops.operator_a(p.op, p.dim, p.n, p.h, eps=p.eps, beta=p.beta)
    out = []
    for n in levels:
        un = U[n - 1].reshape(-1)
        um = (u0 if n == 1 else U[n - 2]).reshape(-1)
        out.append(-((un - um) / p.dt + a @ (p.theta * un + (1.0 - p.theta) * um)))
    return np.array(out).reshape((len(levels),) + U.shape[1:])


def residual_ch(p, U: np.ndarray, u0: np.ndarray, levels=None) -> np.ndarray:
    """True alpha = 0 residual r = -G(U) of the nonlinear CH all-at-once system.

    op == "ch"     : G from eq. nonlinear_G: (C1^(0) (x) I)U - (I (x) Lap_h) U^3
                     + (I (x) Lap_h) U + eps^2 (I (x) Lap_h^2) U - b
    op == "ch_eyre": G from eq. nonlinear_Q: the term (I (x) Lap_h) U is replaced
                     by (C3^(0) (x) Lap_h) U, and b_0 carries (I/dt - Lap_h) u0.
    Evaluated per time level (1-based ``levels``; all levels if None).
    """
    lap = ops.laplacian(p.dim, p.n, p.h)
    e2 = p.eps * p.eps
    if levels is None:
        levels = range(1, p.nt + 1)
    out = []
    for n in levels:
        un = U[n - 1].reshape(-1)
        um = (u0 if n == 1 else U[n - 2]).reshape(-1)
        if p.op == "ch":
            g = (un - um) / p.dt - lap @ (un ** 3) + lap @ un + e2 * (lap @ (lap @ un))
        elif p.op == "ch_eyre":
            g = (un - um) / p.dt - lap @ (un ** 3) + lap @ um + e2 * (lap @ (lap @ un))
        else:
            raise ValueError(p.op)
        out.append(-g)
    return np.array(out).reshape((len(list(levels)),) + U.shape[1:])


def residual(p, U: np.ndarray, u0: np.ndarray) -> np.ndarray:
    """True residual for any operator (all levels)."""
    if p.op in ("biharmonic", "linear_ch"):
        return residual_linear(p, U, u0)
    return residual_ch(p, U, u0)


def mean_jacobian(U: np.ndarray) -> float:
    """Scalar averaged Jacobian c_bar = mean over all space-time points of 3 u^2
    (eq. approx_jacobian, time average of J_s, further averaged in space)."""
    return float(np.mean(3.0 * U * U))


# ------------------------------------------------------------ preconditioner
def precond_matrix(p, c_bar: float = 0.0) -> sp.csr_matrix:
    """The alpha-circulant space-time matrix P_alpha that one outer step inverts.

    linear (biharmonic, linear_ch): C1^(a) (x) I + C2^(a) (x) A         (eq. all-at-once1)
    ch (PinT-I)    : C1^(a) (x) I + (1 - c_bar) (I (x) Lap_h) + eps^2 (I (x) Lap_h^2)
                     (eq. approx_jacobian with J~ = c_bar I)
    ch_eyre (PinT-II): C1^(a) (x) I - c_bar (I (x) Lap_h) + C3^(a) (x) Lap_h
                     + eps^2 (I (x) Lap_h^2)                              (eq. approx_jacoQ)
    """
    if p.op in ("biharmonic", "linear_ch"):
        a = ops.operator_a(p.op, p.dim, p.n, p.h, eps=p.eps, beta=p.beta)
        return allatonce_matrix(a, p.nt, p.dt, p.theta, p.alpha)
    lap = ops.laplacian(p.dim, p.n, p.h)
    lap2 = (lap @ lap).tocsr()
    eye_s = sp.identity(lap.shape[0], format="csr")
    c1, _ = circulant_blocks(p.nt, p.dt, 1.0, p.alpha)
    eye_t = sp.identity(p.nt, format="csr")
    m = sp.kron(sp.csr_matrix(c1), eye_s) + p.eps ** 2 * sp.kron(eye_t, lap2)
    if p.op == "ch":
        m = m + (1.0 - c_bar) * sp.kron(eye_t, lap)
    elif p.op == "ch_eyre":
        m = m - c_bar * sp.kron(eye_t, lap) + sp.kron(sp.csr_matrix(c3_block(p.nt, p.alpha)), lap)
    else:
        raise ValueError(p.op)
    return m.tocsr()


def jacobian_field(U: np.ndarray) -> np.ndarray:
    """The time-averaged Jacobian of the cubic term as the paper defines it
    (eq. approx_jacobian): (1/N_t) sum_n J_s(u_n) with J_s(u) = diag(3 u^2), a
    diagonal that still varies in space; returned as the field of its
    diagonal entries (the shape of one level)."""
    return np.mean(3.0 * U * U, axis=0)


def precond_matrix_field(p, jfield: np.ndarray) -> sp.csr_matrix:
    """The approximate Jacobian of eq. approx_jacobian (PinT-I) with the
    space-varying averaged Jacobian J~ = diag(jfield):
        C1^(a) (x) I - I (x) Lap_h J~ + I (x) Lap_h + eps^2 (I (x) Lap_h^2),
    whose Step-(2) systems (eq. pintiter_CH) lam_{1,l} I - Lap_h J~ + Lap_h +
    eps^2 Lap_h^2 are not diagonal in the cosine basis."""
    if p.op != "ch":
        raise ValueError("the space-varying averaged Jacobian is built for PinT-I")
    lap = ops.laplacian(p.dim, p.n, p.h)
    lap2 = (lap @ lap).tocsr()
    k = (-(lap @ sp.diags(np.asarray(jfield, dtype=np.float64).reshape(-1))) + lap + p.eps ** 2 * lap2).tocsr()
    c1, _ = circulant_blocks(p.nt, p.dt, 1.0, p.alpha)
    eye_s = sp.identity(lap.shape[0], format="csr")
    eye_t = sp.identity(p.nt, format="csr")
    return (sp.kron(sp.csr_matrix(c1), eye_s) + sp.kron(eye_t, k)).tocsr()


def precond_solve_field(p, r: np.ndarray, jfield: np.ndarray) -> np.ndarray:
    """delta = G~'^{-1} r with the space-varying averaged Jacobian, by a sparse
    direct solve (small sizes only)."""
    m = precond_matrix_field(p, jfield).tocsc()
    return spla.spsolve(m, r.reshape(-1)).reshape(r.shape)


def precond_solve(p, r: np.ndarray, c_bar: float = 0.0) -> np.ndarray:
    """delta = P_alpha^{-1} r by a sparse direct (SuperLU) solve.  For small
    space-time sizes only."""
    m = precond_matrix(p, c_bar).tocsc()
    return spla.spsolve(m, r.reshape(-1)).reshape(r.shape)


def dct2_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix from its cosine definition:
    Q[k, j] = s_k cos(pi k (2j+1) / (2n)), s_0 = sqrt(1/n), s_k = sqrt(2/n).
    Its rows are the eigenvectors of the cell-centred Neumann Laplacian."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    # cos has period 4n in the integer k (2j+1): reduce it exactly first, so
    # the argument stays below 2 pi and carries no rounding of order k j u
    m = (k * (2 * j + 1)) % (4 * n)
    q = np.cos(np.pi * m / (2.0 * n)) * np.sqrt(2.0 / n)
    q[0, :] = np.sqrt(1.0 / n)
    return q


def dct2(x: np.ndarray, dim: int) -> np.ndarray:
    """Orthonormal DCT-II over the last ``dim`` axes by dense matrix products
    (2D: Q_y X Q_x^T per slice)."""
    n = x.shape[-1]
    q = dct2_matrix(n)
    y = x @ q.T
    if dim == 2:
        y = np.swapaxes(np.swapaxes(y, -1, -2) @ q.T, -1, -2)
    return y


def idct2(x: np.ndarray, dim: int) -> np.ndarray:
    """Inverse of ``dct2`` (the orthonormal DCT-III): multiplication by Q^T."""
    n = x.shape[-1]
    q = dct2_matrix(n)
    y = x @ q
    if dim == 2:
        y = np.swapaxes(np.swapaxes(y, -1, -2) @ q, -1, -2)
    return y


def spatial_symbols(p, c_bar: float = 0.0):
    """Eigenvalues (per cosine mode, flattened [y][x]) of the spatial operators:
    lam (Laplacian) and mu (of A, linear ops).  Derived from the explicit
    cosine eigenvectors (Lap_h q_k = lam_k q_k for the rows of dct2_matrix)."""
    lam1 = ops.spectrum_1d(p.n, p.h)
    if p.dim == 1:
        lam = lam1
    else:
        lam = (lam1[:, None] + lam1[None, :]).reshape(-1)
    if p.op == "biharmonic":
        mu = lam * lam
    elif p.op == "linear_ch":
        mu = p.beta ** 2 * lam + p.eps ** 2 * lam * lam
    else:
        mu = None
    return lam, mu


def time_solve_modal(p, rh: np.ndarray, c_bar: float = 0.0) -> np.ndarray:
    """The space-time solve in the cosine basis: for each spatial mode k the
    dense N_t x N_t alpha-circulant system (C1 + mu_k C2) y = x (linear), or
    its CH forms, solved by numpy.linalg.solve.  rh is [N_t][modes...] (DCT
    coefficients); returns the same shape."""
    nt = p.nt
    x = rh.reshape(nt, -1)
    lam, mu = spatial_symbols(p)
    c1, c2 = circulant_blocks(nt, p.dt, p.theta if p.op in ("biharmonic", "linear_ch") else 1.0, p.alpha)
    if p.op in ("biharmonic", "linear_ch"):
        mats = c1[None] + mu[:, None, None] * c2[None]
    elif p.op == "ch":
        mats = c1[None] + ((1.0 - c_bar) * lam + p.eps ** 2 * lam * lam)[:, None, None] * np.eye(nt)[None]
    elif p.op == "ch_eyre":
        c3 = c3_block(nt, p.alpha)
        mats = (c1[None] + ((p.eps ** 2 * lam * lam - c_bar * lam)[:, None, None]) * np.eye(nt)[None]
                + lam[:, None, None] * c3[None])
    else:
        raise ValueError(p.op)
    sol = np.linalg.solve(mats, x.T[:, :, None])[:, :, 0]   # [modes][nt]
    return sol.T.reshape(rh.shape)


def time_solve_steps_modal(p, rh: np.ndarray, dts, c_bar: float = 0.0) -> np.ndarray:
    """The space-time solve with nonuniform steps in the cosine basis: per
    spatial mode k the dense N_t x N_t system (B + mu_k C) y = x of the linear
    theta-method (B, C from ``step_blocks``; C = I for backward Euler), or
    (B + ((1 - c_bar) lam_k + eps^2 lam_k^2) I) y = x (backward-Euler CH with
    the scalar averaged Jacobian), solved by numpy.linalg.solve -- no
    eigendecomposition."""
    nt = p.nt
    x = rh.reshape(nt, -1)
    lam, mu = spatial_symbols(p)
    linear = p.op in ("biharmonic", "linear_ch")
    b, c = step_blocks(dts, p.theta if linear else 1.0)
    if linear:
        shift = mu
    elif p.op == "ch":
        shift = (1.0 - c_bar) * lam + p.eps ** 2 * lam * lam
    else:
        raise ValueError(p.op)
    mats = b[None] + shift[:, None, None] * c[None]
    sol = np.linalg.solve(mats, x.T[:, :, None])[:, :, 0]
    return sol.T.reshape(rh.shape)


def precond_solve_modal(p, r: np.ndarray, c_bar: float = 0.0) -> np.ndarray:
    """delta = P_alpha^{-1} r, with the spatial operator diagonalized by the
    explicit orthonormal cosine matrix and one dense N_t x N_t alpha-circulant
    solve per spatial mode (``time_solve_modal``).  Same result as
    ``precond_solve``; usable at moderate sizes."""
    return idct2(time_solve_modal(p, dct2(r, p.dim), c_bar), p.dim)


# ------------------------------------------------------------ outer iteration
def outer_iterate(p, u0: np.ndarray, U: np.ndarray, iters: int, modal: bool = True):
    """Waveform relaxation + one quasi-Newton step per sweep, in correction form:
    U <- U + P_alpha^{-1} r(U) (Sections 2.1 and 4.1, eqs. pintiter1 and
    pintiter_CH with the alpha terms of b^{k-1} cancelled).  Returns the list
    of iterates U^1..U^iters."""
    solve = precond_solve_modal if modal else precond_solve
    U = U.copy()
    hist = []
    for _ in range(iters):
        r = residual(p, U, u0)
        c_bar = mean_jacobian(U) if p.op in ("ch", "ch_eyre") else 0.0
        U = U + solve(p, r, c_bar)
        hist.append(U.copy())
    return hist


def wr_paper_form(p, u0: np.ndarray, U: np.ndarray, iters: int):
    """The paper's linear WR as printed: solve P_alpha U^k = b^{k-1}, with
    b^{k-1} built from u0 - alpha u_{N_t}^{k-1} (eq. all-at-once1)."""
    a = ops.operator_a(p.op, p.dim, p.n, p.h, eps=p.eps, beta=p.beta)
    m = allatonce_matrix(a, p.nt, p.dt, p.theta, p.alpha).tocsc()
    lu = spla.splu(m)
    U = U.copy()
    hist = []
    for _ in range(iters):
        b = rhs_linear(u0, a, p.nt, p.dt, p.theta, p.alpha, U[-1])
        U = lu.solve(b).reshape(U.shape)
        hist.append(U.copy())
    return hist
