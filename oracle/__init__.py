"""CPU FP64 correctness oracle for the all-at-once space-time solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path (no DCT, no FFT,
no diagonalization): the answer it produces is the solution of the sequential,
fully discrete scheme, which the parallel-in-time iteration reaches exactly at
convergence (the alpha-terms of the periodic-like initial condition cancel,
Section 2, eq. modelproblem1a_wr and Section 4, eq. modelproblem3_wr).

Modules
-------
operators   cell-centred Neumann Laplacian, the fourth-order operators, mass
            and the Ginzburg-Landau energy (Sections 1-4).
stepper     sequential theta-method / backward-Euler / Eyre time stepping with
            direct banded (LAPACK Cholesky) spatial solves.
allatonce   the all-at-once matrices (Strang-type alpha-circulant blocks), the
            true alpha=0 residual, direct application of the alpha-circulant
            preconditioner, the orthonormal DCT-II matrix from its cosine
            definition, and the WR / quasi-Newton iteration in correction form.

Readings of the paper that the oracle fixes (grid, eigenvalue convention,
scalar averaged Jacobian ...) are listed in the module docstrings where they
apply.  Parity status: every function is pinned by a ``-m "not gpu"`` test
under ``tests/`` against closed forms, brute force, identities or invariants,
except where a docstring says "parity unpinned".
"""
from . import operators, stepper, allatonce  # noqa: F401
