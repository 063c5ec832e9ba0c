"""PyTorch-facing solver: torch supplies device memory and the stream; the
solve itself runs in the HIP library (include/pint.h)."""
from __future__ import annotations

import torch

from . import _pint


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2304_14021_amd needs a ROCm GPU (gfx950); none is visible")


class Solver:
    """A plan for one problem shape plus its device workspace.

    Parameters follow the paper's problem statement: operator ("biharmonic",
    "linear_ch", "ch", "ch_eyre"), dimension, cells per dimension n, time
    levels nt, step dt, theta, eps, beta, PinT parameter alpha (0 = automatic),
    precision ("fp64"; "fp32": FP32 transforms with FP64 refinement; "mixed":
    FP64 forward spatial transform, FP32 time solve and inverse transform,
    FP64 refinement),
    relative tolerance and iteration cap.
    """

    def __init__(self, op: str, dim: int, n: int, nt: int, dt: float, theta: float = 1.0, eps: float = 1.0,
                 beta: float = 0.0, alpha: float = 1e-3, precision: str = "fp32", time_path: str = "auto",
                 rtol: float = 1e-10, max_iter: int = 30, broadcast_u0: bool = True, stage_timing: bool = False,
                 graph: bool = False, invariants: bool = False, dts=None, field_jacobian: bool = False,
                 device=None):
        _require_gpu()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        flags = (_pint.FLAG_INIT_BROADCAST_U0 if broadcast_u0 else 0) | (_pint.FLAG_STAGE_TIMING if stage_timing else 0)
        # graph: replay init + predicted iterations as one captured HIP graph
        # (needs a non-default torch stream; on the default stream it is ignored)
        flags |= _pint.FLAG_SOLVE_GRAPH if graph else 0
        # invariants: the report carries the mass drift and energy monotonicity
        flags |= _pint.FLAG_INVARIANTS if invariants else 0
        # field_jacobian: the space-varying averaged Jacobian with an inner Krylov solve (CH only)
        flags |= _pint.FLAG_FIELD_JACOBIAN if field_jacobian else 0
        self.shape = (nt,) + (n,) * dim
        self.slice_shape = (n,) * dim
        self.dof = nt * n ** dim
        with torch.cuda.device(self.device):
            self.plan = _pint.Plan(_pint.make_problem(op, dim, n, nt, dt, theta=theta, eps=eps, beta=beta,
                                                      alpha=alpha, precision=precision, time_path=time_path,
                                                      rtol=rtol, max_iter=max_iter, flags=flags, dts=dts))
            self.work = torch.empty(self.plan.work_bytes + 256, dtype=torch.uint8, device=self.device)
        self.alpha = self.plan.alpha

    @classmethod
    def for_problem(cls, p, **kw):
        """Build from any object with the fields op, dim, n, nt, dt, theta, eps, beta, alpha.  A problem
        with nonuniform steps (a field q != 1) needs its steps passed as dts=."""
        if getattr(p, "q", 1.0) != 1.0 and kw.get("dts") is None:
            raise ValueError("a problem with nonuniform steps needs dts=")
        return cls(p.op, p.dim, p.n, p.nt, p.dt, theta=p.theta, eps=p.eps, beta=p.beta, alpha=p.alpha, **kw)

    def _work_ptr(self):
        p = self.work.data_ptr()
        return p + ((-p) % 256)

    def _wdt(self):
        return torch.float64 if self.plan.problem.precision == _pint.PRECISIONS["fp64"] else torch.float32

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def _check(self, t: torch.Tensor, shape, name):
        if t.device != self.device or t.dtype != torch.float64 or tuple(t.shape) != tuple(shape) \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on {self.device}")

    def solve(self, u0: torch.Tensor, U: torch.Tensor | None = None, raise_on_error: bool = True):
        """Solve for u_1..u_nt.  u0: [n]*dim float64 on the device.  U (optional):
        initial guess / output [nt, n, ...] (ignored as a guess when the plan
        broadcasts u0).  Returns (U, report dict)."""
        self._check(u0, self.slice_shape, "u0")
        if U is None:
            U = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check(U, self.shape, "U")
        ok = (_pint.PINT_OK,) if raise_on_error else (_pint.PINT_OK, _pint.PINT_ENOCONV, _pint.PINT_EDIVERGED)
        rep = self.plan.solve_raw(u0.data_ptr(), U.data_ptr(), self._work_ptr(), self.plan.work_bytes,
                                  self._stream(), raise_on=ok)
        return U, _pint.report_dict(rep)

    # ---- stage calls (same kernels as the solve) ----
    def residual(self, u0: torch.Tensor, U: torch.Tensor) -> torch.Tensor:
        self._check(u0, self.slice_shape, "u0")
        self._check(U, self.shape, "U")
        r = torch.empty_like(U)
        self.plan.residual_raw(u0.data_ptr(), U.data_ptr(), r.data_ptr(), self._work_ptr(), self.plan.work_bytes,
                               self._stream())
        return r

    def dct(self, x: torch.Tensor, inverse: bool = False) -> torch.Tensor:
        wdt = self._wdt()
        if x.dtype != wdt or tuple(x.shape) != self.shape or not x.is_contiguous():
            raise ValueError(f"x must be contiguous {wdt} of shape {self.shape}")
        y = torch.empty_like(x)
        self.plan.dct_raw(x.data_ptr(), y.data_ptr(), inverse, self._stream())
        return y

    def time_solve(self, S: torch.Tensor, c_bar: float = 0.0) -> torch.Tensor:
        wdt = self._wdt()
        if S.dtype != wdt or tuple(S.shape) != self.shape or not S.is_contiguous():
            raise ValueError(f"S must be contiguous {wdt} of shape {self.shape}")
        S = S.clone()
        self.plan.time_solve_raw(S.data_ptr(), c_bar, self._stream())
        return S

    def precond(self, r: torch.Tensor, c_bar: float = 0.0) -> torch.Tensor:
        self._check(r, self.shape, "r")
        d = torch.empty_like(r)
        self.plan.precond_raw(r.data_ptr(), d.data_ptr(), c_bar, self._work_ptr(), self.plan.work_bytes,
                              self._stream())
        return d

    def field_jacobian_solve(self, u0: torch.Tensor, U: torch.Tensor, r: torch.Tensor, inner_rtol: float = 1e-12,
                             inner_max: int = 60):
        """(delta, inner iterations): delta = G~'(U)^{-1} r with the space-varying
        averaged Jacobian of U (plans built with field_jacobian=True)."""
        self._check(u0, self.slice_shape, "u0")
        self._check(U, self.shape, "U")
        self._check(r, self.shape, "r")
        d = torch.empty_like(r)
        it = self.plan.field_jacobian_solve_raw(u0.data_ptr(), U.data_ptr(), r.data_ptr(), d.data_ptr(), inner_rtol,
                                                inner_max, self._work_ptr(), self.plan.work_bytes, self._stream())
        return d, it

    def time_eig(self):
        """(V, W, d): the plan's FP64 eigendecomposition of the time-step
        pencil (nonuniform steps only), B V = C V diag(d), W C V = I."""
        return self.plan.time_eig()

    def diagnostics(self, U: torch.Tensor):
        self._check(U, self.shape, "U")
        m = torch.empty(self.shape[0], dtype=torch.float64, device=self.device)
        e = torch.empty_like(m)
        self.plan.diagnostics_raw(U.data_ptr(), m.data_ptr(), e.data_ptr(), self._stream())
        return m, e
