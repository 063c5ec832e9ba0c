"""MI355X (gfx950) all-at-once space-time solver for the fourth-order problems
of Garai & Mandal's diagonalization-based parallel-in-time method.

The hot path is the HIP library ``libpint.so`` (C ABI in include/pint.h);
this package only marshals arguments to it.
"""
from ._pint import PintError, lib  # noqa: F401
from .solver import Solver  # noqa: F401
from .server import Server  # noqa: F401
