"""Pins of the oracle's spatial operators (CPU only).

Each check is an identity fixed by the mathematics, not a re-typing of the
oracle's formula: symmetry and zero row sums of the Neumann Laplacian, the
cosine modes as eigenvectors against LAPACK's symmetric eigensolver, the 2D
Kronecker-sum spectrum (Section 2.2 remark) and the reduction of the linearized
CH operator to the biharmonic one for beta = 0, eps = 1.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import operators as ops
from oracle import allatonce as aao


@pytest.mark.parametrize("dim,n", [(1, 7), (1, 16), (2, 5), (2, 8)])
def test_laplacian_symmetric_conservative(dim, n):
    lap = ops.laplacian(dim, n, 1.0 / n).toarray()
    assert np.allclose(lap, lap.T, atol=0, rtol=0)
    # 1^T Lap_h = 0: the discrete mass is conserved by any Lap_h(.) flux form
    assert np.max(np.abs(lap.sum(axis=0))) < 1e-9 * n * n


@pytest.mark.parametrize("n", [4, 9, 32])
def test_cosine_modes_are_eigenvectors_1d(n):
    h = 1.0 / n
    lap = ops.laplacian_1d(n, h).toarray()
    # brute force: LAPACK eigenvalues of the explicit matrix
    ev = np.sort(sla.eigvalsh(lap))
    # closed form, written independently of the operator code
    k = np.arange(n)
    closed = np.sort(2.0 / h ** 2 * (np.cos(k * np.pi / n) - 1.0))
    assert np.allclose(ev, closed, rtol=1e-12, atol=1e-9)
    # each sampled cosine cos(k pi x_j), x_j = (j + 1/2) h, is an eigenvector
    x = (np.arange(n) + 0.5) * h
    for kk in range(n):
        v = np.cos(kk * np.pi * x)
        lam = 2.0 / h ** 2 * (np.cos(kk * np.pi / n) - 1.0)
        assert np.allclose(lap @ v, lam * v, atol=1e-9 * n * n)


def test_dct_matrix_orthonormal_and_diagonalizes():
    n = 12
    q = aao.dct2_matrix(n)
    assert np.allclose(q @ q.T, np.eye(n), atol=1e-14)
    lap = ops.laplacian_1d(n, 1.0 / n).toarray()
    d = q @ lap @ q.T
    off = d - np.diag(np.diag(d))
    assert np.max(np.abs(off)) < 1e-10 * n * n
    assert np.allclose(np.diag(d), ops.spectrum_1d(n, 1.0 / n), rtol=1e-12, atol=1e-9)


def test_dct_matches_library_routine():
    # special case reducing to a library routine: scipy's orthonormal DCT-II
    import scipy.fft as sfft
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 10, 10))
    assert np.allclose(aao.dct2(x, 2), sfft.dctn(x, type=2, norm="ortho", axes=(1, 2)), atol=1e-13)
    assert np.allclose(aao.idct2(aao.dct2(x, 2), 2), x, atol=1e-13)
    y = rng.standard_normal((4, 16))
    assert np.allclose(aao.dct2(y, 1), sfft.dct(y, type=2, norm="ortho", axis=-1), atol=1e-13)


def test_2d_spectrum_kronecker_sum():
    n = 6
    h = 1.0 / n
    lap = ops.laplacian(2, n, h).toarray()
    ev = np.sort(sla.eigvalsh(lap))
    lam = 2.0 / h ** 2 * (np.cos(np.arange(n) * np.pi / n) - 1.0)
    closed = np.sort((lam[:, None] + lam[None, :]).ravel())
    assert np.allclose(ev, closed, rtol=1e-12, atol=1e-8)


def test_linear_ch_reduces_to_biharmonic():
    n = 8
    a1 = ops.operator_a("biharmonic", 2, n, 1.0 / n).toarray()
    a2 = ops.operator_a("linear_ch", 2, n, 1.0 / n, eps=1.0, beta=0.0).toarray()
    assert np.array_equal(a1, a2)


def test_biharmonic_symbol_and_spinodal_minimum():
    # A = beta^2 Lap + eps^2 Lap^2 has eigenvalues beta^2 lam + eps^2 lam^2
    # whose minimum over lam <= 0 is -beta^4/(4 eps^2) (Section 3)
    n, beta, eps = 64, 0.5, 0.05
    a = ops.operator_a("linear_ch", 1, n, 1.0 / n, eps=eps, beta=beta).toarray()
    ev = sla.eigvalsh(a)
    assert ev.min() >= -beta ** 4 / (4 * eps ** 2) - 1e-9
    assert ev.min() < 0.0


def test_energy_two_forms_agree_and_mass():
    rng = np.random.default_rng(3)
    n, eps = 9, 0.07
    h = 1.0 / n
    u = rng.uniform(-1, 1, (n, n))
    lap = ops.laplacian(2, n, h)
    # summation by parts: sum over faces of squared differences = -u^T Lap_h u * h^2
    alt = h ** 2 * (np.sum(0.25 * (u ** 2 - 1) ** 2) - 0.5 * eps ** 2 * (u.ravel() @ (lap @ u.ravel())))
    assert abs(ops.energy(u, eps, h) - alt) < 1e-12 * abs(alt)
    assert abs(ops.mass(u, h) - h * h * u.sum()) < 1e-15
    # constant state: energy is the bulk term only
    c = np.full((n, n), 0.3)
    assert abs(ops.energy(c, eps, h) - 0.25 * (0.09 - 1) ** 2) < 1e-14
