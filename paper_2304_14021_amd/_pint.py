"""ctypes binding of the C ABI declared in include/pint.h (argument
marshalling only; every step of the solve runs in the HIP library)."""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpint.so")

PINT_OK = 0
PINT_EINVAL = -1
PINT_ENOCONV = -2
PINT_EDIVERGED = -3
PINT_ENOMEM = -4
PINT_EHIP = -5
PINT_ETIMEDOUT = -6
PINT_ECANCELED = -7
PINT_ENOTFOUND = -8

OPS = {"biharmonic": 0, "linear_ch": 1, "ch": 2, "ch_eyre": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_norefine": 2, "bf16": 3, "mixed": 4, "bf16x3": 3, "bf16_norefine": 5}
TIME_PATHS = {"auto": 0, "fft": 1, "dense": 2}
FLAG_INIT_BROADCAST_U0 = 0x1
FLAG_STAGE_TIMING = 0x2
FLAG_BF16_SPLIT = 0x4
FLAG_SOLVE_GRAPH = 0x8
FLAG_INVARIANTS = 0x10
FLAG_FIELD_JACOBIAN = 0x20
HIST = 64

# Every symbol include/pint.h declares (checked by the CPU test suite).
EXPORTS = (
    "pint_status_string", "pint_last_error", "pint_version",
    "pint_plan_create", "pint_plan_destroy", "pint_plan_last_error", "pint_plan_workspace_size",
    "pint_plan_alpha", "pint_solve", "pint_solve_noalloc", "pint_residual", "pint_dct", "pint_time_solve",
    "pint_precond_apply", "pint_diagnostics", "pint_time_eig", "pint_field_jacobian_solve",
    "pint_server_create", "pint_server_submit", "pint_server_submit_device", "pint_server_wait", "pint_server_cancel", "pint_server_stats",
    "pint_server_destroy", "pint_server_last_error",
)
SERVER_NO_GRAPHS = 0x1


class Problem(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_size_t),
        ("op", ct.c_int), ("dim", ct.c_int), ("nx", ct.c_int), ("ny", ct.c_int), ("nt", ct.c_int),
        ("lx", ct.c_double), ("ly", ct.c_double),
        ("dt", ct.c_double), ("theta", ct.c_double), ("eps", ct.c_double), ("beta", ct.c_double),
        ("alpha", ct.c_double),
        ("precision", ct.c_int), ("time_path", ct.c_int),
        ("rtol", ct.c_double), ("max_iter", ct.c_int), ("flags", ct.c_uint),
        ("dts", ct.POINTER(ct.c_double)),
    ]


class Report(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_size_t),
        ("status", ct.c_int), ("iterations", ct.c_int),
        ("alpha_used", ct.c_double), ("c_bar", ct.c_double), ("est_rel_err", ct.c_double),
        ("res_hist", ct.c_double * HIST), ("upd_hist", ct.c_double * HIST),
        ("ms_stage", ct.c_double * 8), ("ms_total", ct.c_double),
        ("mass_drift", ct.c_double), ("energy_monotone", ct.c_int), ("inner_iterations", ct.c_int),
    ]


class ServerConfig(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_size_t), ("d_pool", ct.c_void_p), ("pool_bytes", ct.c_size_t),
        ("max_active", ct.c_int), ("flags", ct.c_uint), ("host_pool_bytes", ct.c_size_t),
    ]


class ServerStats(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_size_t),
        ("submitted", ct.c_uint64), ("completed", ct.c_uint64), ("failed", ct.c_uint64), ("cancelled", ct.c_uint64),
        ("queued", ct.c_int), ("active", ct.c_int),
        ("pool_bytes", ct.c_size_t), ("pool_in_use", ct.c_size_t), ("pool_peak", ct.c_size_t),
        ("p50_ms", ct.c_double), ("p99_ms", ct.c_double), ("mean_ms", ct.c_double), ("max_ms", ct.c_double),
        ("dof_completed", ct.c_double), ("busy_seconds", ct.c_double),
        ("graphs_captured", ct.c_uint64), ("graph_updates", ct.c_uint64), ("graph_launches", ct.c_uint64),
        ("worker_host_seconds", ct.c_double),
        ("host_pool_bytes", ct.c_size_t), ("host_pool_in_use", ct.c_size_t),
    ]


class PintError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Lib:
    """Thin wrapper over one loaded copy of the library."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            raise RuntimeError(
                f"HIP library not built: {path} is missing (run __graft_entry__.build() or "
                "python -m paper_2304_14021_amd.build)")
        self.path = path
        self.dll = ct.CDLL(path)
        d = self.dll
        vp, i, dbl, sz = ct.c_void_p, ct.c_int, ct.c_double, ct.c_size_t
        d.pint_status_string.restype = ct.c_char_p
        d.pint_status_string.argtypes = [i]
        d.pint_last_error.restype = ct.c_char_p
        d.pint_version.restype = ct.c_char_p
        d.pint_plan_create.argtypes = [ct.POINTER(Problem), ct.POINTER(vp)]
        d.pint_plan_destroy.argtypes = [vp]
        d.pint_plan_last_error.restype = ct.c_char_p
        d.pint_plan_last_error.argtypes = [vp]
        d.pint_plan_workspace_size.argtypes = [vp, ct.POINTER(sz)]
        d.pint_plan_alpha.argtypes = [vp, ct.POINTER(dbl)]
        d.pint_solve.argtypes = [vp, vp, vp, vp, sz, vp, ct.POINTER(Report)]
        d.pint_solve_noalloc.argtypes = [vp, vp, vp, vp, ct.POINTER(Report)]
        d.pint_residual.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        d.pint_dct.argtypes = [vp, vp, vp, i, vp]
        d.pint_time_solve.argtypes = [vp, vp, dbl, vp]
        d.pint_precond_apply.argtypes = [vp, vp, vp, dbl, vp, sz, vp]
        d.pint_diagnostics.argtypes = [vp, vp, vp, vp, vp]
        d.pint_time_eig.argtypes = [vp, vp, vp, vp]
        d.pint_field_jacobian_solve.argtypes = [vp, vp, vp, vp, vp, dbl, i, vp, sz, vp, ct.POINTER(i)]
        d.pint_server_create.argtypes = [ct.POINTER(ServerConfig), ct.POINTER(vp)]
        d.pint_server_submit.argtypes = [vp, ct.POINTER(Problem), vp, ct.POINTER(ct.c_uint64)]
        d.pint_server_submit_device.argtypes = [vp, ct.POINTER(Problem), vp, vp, ct.POINTER(ct.c_uint64)]
        d.pint_server_wait.argtypes = [vp, ct.c_uint64, vp, ct.POINTER(Report), i]
        d.pint_server_cancel.argtypes = [vp, ct.c_uint64]
        d.pint_server_stats.argtypes = [vp, ct.POINTER(ServerStats)]
        d.pint_server_destroy.argtypes = [vp]
        d.pint_server_last_error.restype = ct.c_char_p
        d.pint_server_last_error.argtypes = [vp]
        for name in EXPORTS:
            if name not in ("pint_status_string", "pint_last_error", "pint_version", "pint_plan_last_error",
                            "pint_server_last_error"):
                getattr(d, name).restype = ct.c_int

    def check(self, rc: int, plan=None, ok=(PINT_OK,)):
        if rc in ok:
            return rc
        msg = (self.dll.pint_plan_last_error(plan) if plan else self.dll.pint_last_error()) or b""
        raise PintError(rc, msg.decode() or self.dll.pint_status_string(rc).decode())


_LIB = None


def lib() -> Lib:
    """The in-tree HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        _LIB = Lib(LIB_PATH)
    return _LIB


def make_problem(op: str, dim: int, n: int, nt: int, dt: float, theta: float = 1.0, eps: float = 1.0,
                 beta: float = 0.0, alpha: float = 1e-3, precision: str = "fp32", time_path: str = "auto",
                 rtol: float = 1e-10, max_iter: int = 30, flags: int = 0, length: float = 1.0,
                 dts=None) -> Problem:
    """A pint_problem struct.  dts: optional nonuniform steps (nt values); the
    array is kept referenced by the struct (``p._dts``) until it is dropped."""
    p = Problem()
    p.struct_size = ct.sizeof(Problem)
    p.op = OPS[op]
    p.dim = dim
    p.nx = n
    p.ny = n if dim == 2 else 1
    p.nt = nt
    p.lx = p.ly = length
    p.dt = dt
    p.theta = theta
    p.eps = eps
    p.beta = beta
    p.alpha = alpha
    p.precision = PRECISIONS[precision]
    if precision == "bf16x3":  # BF16 with the two-term operand split
        flags |= FLAG_BF16_SPLIT
    p.time_path = TIME_PATHS[time_path]
    p.rtol = rtol
    p.max_iter = max_iter
    p.flags = flags
    if dts is not None:
        import numpy as np
        arr = np.ascontiguousarray(dts, dtype=np.float64)
        if arr.shape != (nt,):
            raise ValueError(f"dts must hold nt = {nt} steps")
        p._dts = arr
        p.dts = arr.ctypes.data_as(ct.POINTER(ct.c_double))
    return p


class Plan:
    """Owns one pint_plan (constant tables on the current device)."""

    def __init__(self, problem: Problem, library: Lib | None = None):
        self.lib = library or lib()
        self.problem = problem
        h = ct.c_void_p()
        self.lib.check(self.lib.dll.pint_plan_create(ct.byref(problem), ct.byref(h)))
        self.h = h
        b = ct.c_size_t()
        self.lib.check(self.lib.dll.pint_plan_workspace_size(self.h, ct.byref(b)), self.h)
        self.work_bytes = b.value
        a = ct.c_double()
        self.lib.check(self.lib.dll.pint_plan_alpha(self.h, ct.byref(a)), self.h)
        self.alpha = a.value

    def close(self):
        if self.h:
            self.lib.dll.pint_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # raw calls: pointers are integers (device addresses), stream an integer handle
    def solve_raw(self, u0_ptr: int, U_ptr: int, work_ptr: int, work_bytes: int, stream: int = 0,
                  raise_on=(PINT_OK,)) -> Report:
        rep = Report()
        rep.struct_size = ct.sizeof(Report)
        rc = self.lib.dll.pint_solve(self.h, u0_ptr, U_ptr, work_ptr, work_bytes, stream, ct.byref(rep))
        self.lib.check(rc, self.h, ok=raise_on)
        return rep

    def residual_raw(self, u0_ptr, U_ptr, r_ptr, work_ptr, work_bytes, stream=0):
        self.lib.check(self.lib.dll.pint_residual(self.h, u0_ptr, U_ptr, r_ptr, work_ptr, work_bytes, stream), self.h)

    def dct_raw(self, in_ptr, out_ptr, inverse: bool, stream=0):
        self.lib.check(self.lib.dll.pint_dct(self.h, in_ptr, out_ptr, 1 if inverse else 0, stream), self.h)

    def time_solve_raw(self, s_ptr, c_bar: float, stream=0):
        self.lib.check(self.lib.dll.pint_time_solve(self.h, s_ptr, c_bar, stream), self.h)

    def precond_raw(self, r_ptr, d_ptr, c_bar, work_ptr, work_bytes, stream=0):
        self.lib.check(self.lib.dll.pint_precond_apply(self.h, r_ptr, d_ptr, c_bar, work_ptr, work_bytes, stream),
                       self.h)

    def field_jacobian_solve_raw(self, u0_ptr, U_ptr, r_ptr, d_ptr, inner_rtol, inner_max, work_ptr, work_bytes,
                                 stream=0) -> int:
        it = ct.c_int()
        self.lib.check(self.lib.dll.pint_field_jacobian_solve(self.h, u0_ptr, U_ptr, r_ptr, d_ptr, inner_rtol,
                                                              inner_max, work_ptr, work_bytes, stream,
                                                              ct.byref(it)), self.h)
        return it.value

    def time_eig(self):
        """(V, W, d) of the plan's FP64 time-step eigendecomposition (host arrays)."""
        import numpy as np
        nt = self.problem.nt
        V, W, d = np.empty((nt, nt)), np.empty((nt, nt)), np.empty(nt)
        self.lib.check(self.lib.dll.pint_time_eig(self.h, V.ctypes.data, W.ctypes.data, d.ctypes.data), self.h)
        return V, W, d

    def diagnostics_raw(self, U_ptr, mass_ptr, energy_ptr, stream=0):
        self.lib.check(self.lib.dll.pint_diagnostics(self.h, U_ptr, mass_ptr, energy_ptr, stream), self.h)


def report_dict(rep: Report) -> dict:
    k = rep.iterations
    return {
        "status": rep.status,
        "iterations": k,
        "alpha": rep.alpha_used,
        "c_bar": rep.c_bar,
        "est_rel_err": rep.est_rel_err,
        "res_hist": list(rep.res_hist[:k]),
        "upd_hist": list(rep.upd_hist[:k]),
        "ms_stage": list(rep.ms_stage[:6]),
        "ms_total": rep.ms_total,
        "mass_drift": rep.mass_drift,
        "energy_monotone": rep.energy_monotone,
        "inner_iterations": rep.inner_iterations,
    }
