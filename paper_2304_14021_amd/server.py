"""Python handle on the library's serving loop (include/pint.h, pint_server_*).

torch supplies the device pool; the persistent worker thread, admission,
streams and graphs live in the HIP library."""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _pint


class Server:
    """A running server with a device pool of ``pool_bytes``, up to
    ``max_active`` requests in flight, and a pinned host pool of
    ``host_pool_bytes`` (0: 1 GiB) for results of host-buffer requests."""

    def __init__(self, pool_bytes: int, max_active: int = 8, graphs: bool = True, device=None,
                 library: _pint.Lib | None = None, host_pool_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a ROCm GPU")
        self.lib = library or _pint.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            self.pool = torch.empty(pool_bytes + 256, dtype=torch.uint8, device=self.device)
            p = self.pool.data_ptr()
            cfg = _pint.ServerConfig()
            cfg.struct_size = ct.sizeof(_pint.ServerConfig)
            cfg.d_pool = p + ((-p) % 256)
            cfg.pool_bytes = pool_bytes
            cfg.max_active = max_active
            cfg.flags = 0 if graphs else _pint.SERVER_NO_GRAPHS
            cfg.host_pool_bytes = host_pool_bytes
            h = ct.c_void_p()
            self._check(self.lib.dll.pint_server_create(ct.byref(cfg), ct.byref(h)), None)
        self.h = h
        self._shapes = {}
        self._held = {}

    def _check(self, rc, h, ok=(_pint.PINT_OK,)):
        if rc in ok:
            return rc
        msg = self.lib.dll.pint_server_last_error(h) or b""
        raise _pint.PintError(rc, msg.decode() or self.lib.dll.pint_status_string(rc).decode())

    @staticmethod
    def _struct(problem, precision, rtol, max_iter):
        if isinstance(problem, _pint.Problem):
            return problem
        p = problem
        return _pint.make_problem(p.op, p.dim, p.n, p.nt, p.dt, theta=p.theta, eps=p.eps, beta=p.beta,
                                  alpha=p.alpha, precision=precision, rtol=rtol, max_iter=max_iter)

    @staticmethod
    def _shape(problem):
        return (problem.nt,) + ((problem.nx,) if problem.dim == 1 else (problem.ny, problem.nx))

    def submit(self, problem, u0: np.ndarray, precision: str = "mixed", rtol: float = 1e-10,
               max_iter: int = 30) -> int:
        """Queue one solve and return its ticket.  ``problem`` is a
        ``pint_problem`` struct, or any object with the fields op, dim, n, nt,
        dt, theta, eps, beta, alpha (then ``precision``, ``rtol`` and
        ``max_iter`` complete it).  u0 is a host array of one time slice; the
        result comes back as a host array from ``wait``."""
        problem = self._struct(problem, precision, rtol, max_iter)
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        ns = problem.nx * (problem.ny if problem.dim == 2 else 1)
        if u0.size != ns:
            raise ValueError(f"u0 has {u0.size} values, the problem's time slice {ns}")
        t = ct.c_uint64()
        self._check(self.lib.dll.pint_server_submit(self.h, ct.byref(problem), u0.ctypes.data, ct.byref(t)), self.h)
        self._shapes[t.value] = self._shape(problem)
        return t.value

    def submit_device(self, problem, u0: torch.Tensor, U: torch.Tensor, precision: str = "mixed",
                      rtol: float = 1e-10, max_iter: int = 30, sync: bool = True) -> int:
        """Device-resident request: u0 ([n]*dim) and U ([nt, n, ...]) are
        contiguous float64 tensors on the server's device; the solve iterates
        in place on U, which holds the result once ``wait`` returns.  Both
        tensors are kept referenced until then.  u0 must hold its values when
        the server reads it: with ``sync`` the current stream is synchronized
        here; pass False when the caller has already synchronized."""
        problem = self._struct(problem, precision, rtol, max_iter)
        shape = self._shape(problem)
        for t, sh, name in ((u0, shape[1:], "u0"), (U, shape, "U")):
            if t.device != self.device or t.dtype != torch.float64 or tuple(t.shape) != sh \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 tensor of shape {sh} on {self.device}")
        if sync:
            torch.cuda.current_stream(self.device).synchronize()
        t = ct.c_uint64()
        self._check(self.lib.dll.pint_server_submit_device(self.h, ct.byref(problem), u0.data_ptr(), U.data_ptr(),
                                                           ct.byref(t)), self.h)
        self._shapes[t.value] = None
        self._held[t.value] = (u0, U)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1, raise_on_error: bool = True):
        """(U, report dict) of a finished request: U is a host array, or the
        caller's device tensor for a device-resident request."""
        shape = self._shapes.get(ticket)
        out = np.empty(shape, dtype=np.float64) if shape else None
        rep = _pint.Report()
        rep.struct_size = ct.sizeof(_pint.Report)
        rc = self.lib.dll.pint_server_wait(self.h, ticket, out.ctypes.data if out is not None else None,
                                           ct.byref(rep), timeout_ms)
        if rc != _pint.PINT_ETIMEDOUT:
            self._shapes.pop(ticket, None)
            held = self._held.pop(ticket, None)
            if held is not None:
                out = held[1]
        ok = (_pint.PINT_OK,) if raise_on_error else (_pint.PINT_OK, _pint.PINT_ENOCONV, _pint.PINT_EDIVERGED,
                                                      _pint.PINT_ECANCELED)
        self._check(rc, self.h, ok=ok)
        d = _pint.report_dict(rep)
        d["status"] = rc
        return out, d

    def cancel(self, ticket: int):
        self._check(self.lib.dll.pint_server_cancel(self.h, ticket), self.h)

    def stats(self) -> dict:
        st = _pint.ServerStats()
        st.struct_size = ct.sizeof(_pint.ServerStats)
        self._check(self.lib.dll.pint_server_stats(self.h, ct.byref(st)), self.h)
        return {name: getattr(st, name) for name, _ in _pint.ServerStats._fields_ if name != "struct_size"}

    def close(self):
        """Shut the server down; raises PintError if a HIP error stopped it or
        surfaced when its streams were synchronized."""
        if getattr(self, "h", None):
            h, self.h = self.h, None
            self._check(self.lib.dll.pint_server_destroy(h), None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
