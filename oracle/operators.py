"""Spatial operators of the oracle (test infrastructure; FP64, SciPy sparse).

Grid reading.  The paper's Laplacian (Section 2.1, eq. deltah) is written on a
vertex-centred grid with boundary rows [-2 2].  The hot path is diagonalized by
the DCT-II, whose eigenvectors belong to the *cell-centred* Neumann Laplacian,
so the oracle uses that one: N cells, h = 1/N, x_j = (j + 1/2) h, and the
homogeneous Neumann condition imposed by ghost reflection u_{-1} = u_0,
u_N = u_{N-1}.  This gives the symmetric matrix tridiag(1, -2, 1)/h^2 with
corner entries -1/h^2.  Its spectrum is (2/h^2)(cos(k pi / N) - 1),
k = 0..N-1, the cell-centred analogue of the spectrum given in Section 2.2.

The fourth-order operators are built by composing the same Laplacian, so the
discrete biharmonic is exactly Lap_h o Lap_h (Section 2.1: A = Lap_h^2), which
also imposes the second Neumann condition d_nu(Lap u) = 0.  In 2D the
Laplacian is the Kronecker sum I (x) L_x + L_y (x) I on row-major [y][x]
arrays (Section 2.2, remark on the 2D spectrum).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplacian_1d(n: int, h: float) -> sp.csr_matrix:
    """Cell-centred Neumann Laplacian on n cells (Section 2.1, eq. deltah,
    cell-centred reading): tridiag(1,-2,1)/h^2 with D[0,0] = D[n-1,n-1] = -1/h^2."""
    main = np.full(n, -2.0)
    main[0] = -1.0
    main[-1] = -1.0
    off = np.ones(n - 1)
    return (sp.diags([off, main, off], [-1, 0, 1], format="csr") / (h * h)).tocsr()


def laplacian(dim: int, n: int, h: float) -> sp.csr_matrix:
    """Discrete Laplacian on the unit interval (dim=1) or square (dim=2,
    row-major [y][x], Kronecker sum I_y (x) L_x + L_y (x) I_x)."""
    d1 = laplacian_1d(n, h)
    if dim == 1:
        return d1
    if dim == 2:
        eye = sp.identity(n, format="csr")
        return (sp.kron(eye, d1) + sp.kron(d1, eye)).tocsr()
    raise ValueError("dim must be 1 or 2")


def operator_a(op: str, dim: int, n: int, h: float, eps: float = 1.0, beta: float = 0.0) -> sp.csr_matrix:
    """The linear fourth-order operator A with u_t + A u = 0.

    biharmonic: A = Lap_h^2                     (Section 2.1, A = Delta_h^2)
    linear_ch : A = beta^2 Lap_h + eps^2 Lap_h^2 (Section 3, eq. modelproblem2a)
    """
    lap = laplacian(dim, n, h)
    lap2 = (lap @ lap).tocsr()
    if op == "biharmonic":
        return lap2
    if op == "linear_ch":
        return (beta * beta * lap + eps * eps * lap2).tocsr()
    raise ValueError(f"no linear operator for op={op!r}")


def spectrum_1d(n: int, h: float) -> np.ndarray:
    """Eigenvalues of laplacian_1d, indexed by the cosine mode k = 0..n-1.
    The eigenvector of mode k is cos(k pi x_j) at the cell centres."""
    k = np.arange(n, dtype=np.float64)
    return (2.0 / (h * h)) * (np.cos(k * np.pi / n) - 1.0)


def mass(u: np.ndarray, h: float) -> float:
    """Discrete mass h^d * sum_j u_j (the integral of u over the domain,
    conserved by the CH equation, Section 1 eq. energy minimization)."""
    return float(h ** u.ndim * np.sum(u))


def energy(u: np.ndarray, eps: float, h: float) -> float:
    """Discrete Ginzburg-Landau energy (Section 1):
    E_h(u) = h^d [ sum_j F(u_j) + (eps^2/2) sum over interior faces ((u_j' - u_j)/h)^2 ],
    F(u) = (u^2 - 1)^2 / 4.  The paper plots the discrete energy without
    defining it; this is the cell-centred finite-volume form of the integral."""
    bulk = np.sum(0.25 * (u * u - 1.0) ** 2)
    grad = 0.0
    for ax in range(u.ndim):
        d = np.diff(u, axis=ax) / h
        grad += np.sum(d * d)
    return float(h ** u.ndim * (bulk + 0.5 * eps * eps * grad))


def f_cubic(u: np.ndarray) -> np.ndarray:
    """f(u) = F'(u) = u^3 - u (Section 1)."""
    return u * u * u - u


def sym_band_upper(m: sp.spmatrix) -> tuple[np.ndarray, int]:
    """Upper banded storage ab[b + i - j, j] = M[i, j] (i <= j) of a symmetric
    sparse matrix, as LAPACK's banded Cholesky expects.  Returns (ab, b)."""
    c = sp.triu(m).tocoo()
    b = int(np.max(c.col - c.row)) if c.nnz else 0
    ab = np.zeros((b + 1, m.shape[0]))
    ab[b + c.row - c.col, c.col] = c.data
    return ab, b
