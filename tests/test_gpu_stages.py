"""Per-stage parity of the HIP kernels against the CPU oracle (GPU).

Stages: a1 residual (FP64 arithmetic), a2/a6 batched orthonormal DCT-II/III,
a3-a5 the alpha-circulant time solve in the cosine basis, and a2-a6 together
(P_alpha^{-1} applied to an FP64 residual).  Sizes span several workgroups
(several time levels, several spatial-mode tiles) for every operator, both
working precisions, 1D and 2D, and the smallest and largest supported sizes.

Tolerances (derived from the arithmetic):
* residual: FP64 on both sides, each entry a short sum of O(1) terms scaled by
  1/dt and 1/h^4: 1e-13 relative to max|r|.
* DCT: orthonormal (the 2-norm of every batch is kept), computed by a radix-8
  FFT of log2(N_s) butterfly levels over the passes, each rounding its outputs
  by about u (u = 2^-53 FP64, 2^-24 FP32) relative to their size, so the error
  of an output is of order u sqrt(log2 N_s) times the RMS of the input.  The
  bound, also for the largest of up to 2^28 outputs (about 6 standard
  deviations): 8 u log2(N_s) x RMS(x), plus 16 u64 sqrt(N) x RMS(x) for the
  oracle's own FP64 dense products (N-term sums).  A twiddle or post-twiddle
  table rounded to BF16 or FP16 (or a wrong entry) exceeds it by orders of
  magnitude.
* time solve / preconditioner: the Gamma_alpha scaling turns an absolute
  rounding error of u * max_j |a^j x_j| at time level j into a relative one
  multiplied by a^{-(N_t-1)} < 1/alpha; the bound used is
  64 u log2(N N_t) / alpha.
"""
import math

import numpy as np
import pytest
import torch

from oracle import allatonce as aao
from paper_2304_14021_amd import Solver
from workloads import Problem
from tests._gpu import dev, host, say, to_dev

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24

CASES = [
    Problem(op="biharmonic", dim=1, n=64, nt=32, dt=1e-3 / 32, alpha=1e-3),
    Problem(op="biharmonic", dim=1, n=8, nt=4, dt=1e-4, alpha=0.05),
    Problem(op="linear_ch", dim=1, n=512, nt=64, dt=1e-6, theta=0.5, eps=0.05, beta=0.5, alpha=0.02),
    Problem(op="linear_ch", dim=2, n=32, nt=64, dt=1e-5, eps=0.05, beta=0.5, alpha=0.01),
    Problem(op="linear_ch", dim=2, n=16, nt=16, dt=1e-5, theta=0.5, eps=0.05, beta=0.5, alpha=0.05),
    Problem(op="biharmonic", dim=2, n=8, nt=8, dt=1e-5, alpha=0.05),
    Problem(op="ch", dim=2, n=64, nt=32, dt=1e-6, eps=0.02, alpha=0.01),
    Problem(op="ch_eyre", dim=2, n=32, nt=16, dt=1e-5, eps=0.05, alpha=0.05),
    Problem(op="linear_ch", dim=2, n=128, nt=16, dt=1e-5, eps=0.05, beta=0.5, alpha=0.05),
    Problem(op="ch", dim=2, n=256, nt=8, dt=1e-6, eps=0.01, alpha=0.05),
    Problem(op="linear_ch", dim=2, n=512, nt=4, dt=1e-6, theta=0.5, eps=0.03, beta=0.4, alpha=0.1),
    Problem(op="biharmonic", dim=1, n=32, nt=1024, dt=1e-6, alpha=0.05),
]
IDS = [f"{p.op}-{p.dim}d-n{p.n}-nt{p.nt}" for p in CASES]


def _solver(p, prec):
    return Solver.for_problem(p, precision=prec, device=dev())


@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_residual_stage(p):
    say(f"residual stage {p}")
    rng = np.random.default_rng(3)
    u0 = rng.uniform(-0.5, 0.5, p.slice_shape)
    U = rng.uniform(-0.5, 0.5, p.shape)
    s = _solver(p, "fp64")
    r = host(s.residual(to_dev(u0), to_dev(U)))
    ref = aao.residual(p, U, u0)
    err = np.max(np.abs(r - ref)) / np.max(np.abs(ref))
    assert err < 1e-13, err


def _idct2(y, dim):
    """Inverse of the oracle's orthonormal DCT-II: the transposed matrix along
    each transformed axis."""
    q = aao.dct2_matrix(y.shape[-1])
    x = y @ q
    if dim == 2:
        x = np.swapaxes(np.swapaxes(x, -1, -2) @ q, -1, -2)
    return x


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_dct_stage(p, prec):
    say(f"dct stage {prec} {p}")
    rng = np.random.default_rng(4)
    x = rng.standard_normal(p.shape)
    s = _solver(p, prec)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    xd = to_dev(x, tdt)
    y = host(s.dct(xd))
    xin = host(xd).astype(np.float64)
    ref = aao.dct2(xin, p.dim)
    u = U64 if prec == "fp64" else U32
    tol = 8 * u * math.log2(p.ns) + 16 * U64 * math.sqrt(p.n)
    rms = float(np.sqrt(np.mean(xin ** 2)))
    ef = np.max(np.abs(y - ref)) / rms
    zin = host(to_dev(ref, tdt)).astype(np.float64)
    z = host(s.dct(to_dev(zin, tdt), inverse=True))
    ei = np.max(np.abs(z - _idct2(zin, p.dim))) / float(np.sqrt(np.mean(zin ** 2)))
    say(f"  forward {ef / u:.2f} u x RMS, inverse {ei / u:.2f} u x RMS (bound {tol / u:.1f} u)")
    assert ef <= tol, ("forward", ef, tol)
    assert ei <= tol, ("inverse", ei, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_time_solve_stage(p, prec):
    say(f"time-solve stage {prec} {p}")
    rng = np.random.default_rng(5)
    xh = rng.standard_normal(p.shape)
    c_bar = 0.37 if p.op in ("ch", "ch_eyre") else 0.0
    s = _solver(p, prec)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    xd = to_dev(xh, tdt)
    y = host(s.time_solve(xd, c_bar))
    ref = aao.time_solve_modal(p, host(xd).astype(np.float64), c_bar)
    u = U64 if prec == "fp64" else U32
    tol = 64 * u * math.log2(p.ns * p.nt) / p.alpha
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    assert err < tol, (err, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stage_buffers_must_be_16_byte_aligned(prec):
    """The DCT and time-solve stages move 16-byte pairs: a buffer 4 or 8
    bytes off a 16-byte boundary is rejected with PINT_EINVAL before any
    launch (the pointer is never dereferenced)."""
    from paper_2304_14021_amd._pint import PINT_EINVAL, PintError
    p = Problem(op="biharmonic", dim=2, n=16, nt=8, dt=1e-4, alpha=0.05)
    say(f"stage alignment check {prec} {p}")
    s = _solver(p, prec)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    buf = torch.zeros(p.nt * p.ns + 4, dtype=tdt, device=dev())
    base = buf.data_ptr()
    assert base % 16 == 0
    off = base + buf.element_size()  # 4 or 8 bytes past the boundary
    for call in (lambda: s.plan.dct_raw(off, base, False), lambda: s.plan.dct_raw(base, off, True),
                 lambda: s.plan.time_solve_raw(off, 0.0)):
        with pytest.raises(PintError) as ei:
            call()
        assert ei.value.code == PINT_EINVAL
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("p", CASES, ids=IDS)
def test_precond_stage(p, prec):
    say(f"precond stage {prec} {p}")
    rng = np.random.default_rng(6)
    r = rng.standard_normal(p.shape)
    c_bar = 0.21 if p.op in ("ch", "ch_eyre") else 0.0
    s = _solver(p, prec)
    d = host(s.precond(to_dev(r), c_bar))
    ref = aao.precond_solve_modal(p, r, c_bar)
    u = U64 if prec == "fp64" else U32
    tol = 64 * u * math.log2(p.ns * p.nt) / p.alpha
    err = np.max(np.abs(d - ref)) / np.max(np.abs(ref))
    assert err < tol, (err, tol)


def test_precond_equals_direct_sparse_solve_small():
    # the modal oracle is itself pinned against a sparse direct solve; check
    # the GPU against the direct solve too on a tiny case
    p = Problem(op="ch", dim=2, n=8, nt=8, dt=1e-5, eps=0.05, alpha=0.05)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(p.shape)
    s = _solver(p, "fp64")
    d = host(s.precond(to_dev(r), 0.3))
    ref = aao.precond_solve(p, r, 0.3)
    assert np.max(np.abs(d - ref)) / np.max(np.abs(ref)) < 1e-11
