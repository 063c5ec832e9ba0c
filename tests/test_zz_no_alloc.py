"""pint_solve_noalloc (the entry point for callers that cannot allocate):
the same solve as pint_solve, with the library's static device workspace.

Checked through the C ABI against pint_solve with a caller workspace, bit for
bit, on two calls in a row (the second on a smaller problem, so the shared
workspace holds the first call's contents), and against the sequential
oracle at the 1e-10 bar (the paper's error norm, Section 5).
"""
import ctypes as ct

import numpy as np
import pytest
import torch

from oracle import stepper
from paper_2304_14021_amd import Solver, _pint
from workloads import Problem
from tests._gpu import dev, host, say, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(p, prec, u0):
    lib = _pint.lib()
    plan = _pint.Plan(_pint.make_problem(p.op, p.dim, p.n, p.nt, p.dt, theta=p.theta, eps=p.eps, beta=p.beta,
                                         alpha=p.alpha, precision=prec,
                                         flags=_pint.FLAG_INIT_BROADCAST_U0))
    d0 = to_dev(u0)
    U = torch.full(p.shape, float("nan"), dtype=torch.float64, device=dev())
    torch.cuda.synchronize()
    rep = _pint.Report()
    rep.struct_size = ct.sizeof(_pint.Report)
    rc = lib.dll.pint_solve_noalloc(plan.h, d0.data_ptr(), U.data_ptr(),
                                    torch.cuda.current_stream(dev()).cuda_stream, ct.byref(rep))
    lib.check(rc, plan.h)
    out = host(U)
    plan.close()
    return out, _pint.report_dict(rep)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_equals_pint_solve_two_calls(prec):
    big = Problem(op="linear_ch", dim=2, n=128, nt=64, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3)
    small = Problem(op="ch", dim=2, n=32, nt=32, dt=1e-6, eps=0.02, alpha=1e-3)
    rng = np.random.default_rng(31)
    for p, amp in ((big, 0.05), (small, 0.3)):
        u0 = rng.uniform(-amp, amp, p.slice_shape)
        say(f"noalloc {prec} {p}")
        U, rep = _noalloc(p, prec, u0)
        s = Solver.for_problem(p, precision=prec, device=dev())
        Ur, rrep = s.solve(to_dev(u0))
        ref = host(Ur)
        err = stepper.rel_err(U, stepper.sequential(p, u0))
        say(f"  iterations {rep['iterations']} (pint_solve {rrep['iterations']}), err vs oracle {err:.2e}")
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, ref)
        assert err <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "fp64", "mixed"])
def test_noalloc_panel_layout(prec):
    # N_t >= 512 in 2D: the spectral array of the time solve is kept in
    # line-wide panels, a second spectral buffer in the static workspace; then
    # a smaller plain-layout call on the same workspace
    first = Problem(op="ch", dim=2, n=16, nt=512, dt=1e-6, eps=0.05, alpha=1e-3)
    second = Problem(op="linear_ch", dim=2, n=16, nt=64, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3)
    rng = np.random.default_rng(37)
    for p, amp in ((first, 0.3), (second, 0.05)):
        u0 = rng.uniform(-amp, amp, p.slice_shape)
        say(f"noalloc {prec} {p}")
        U, rep = _noalloc(p, prec, u0)
        s = Solver.for_problem(p, precision=prec, device=dev())
        Ur, rrep = s.solve(to_dev(u0))
        err = stepper.rel_err(U, stepper.sequential(p, u0))
        say(f"  iterations {rep['iterations']} (pint_solve {rrep['iterations']}), err vs oracle {err:.2e}")
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, host(Ur))
        assert err <= 1e-10


def test_noalloc_rejects_too_large_and_flags():
    lib = _pint.lib()
    p = _pint.make_problem("linear_ch", 2, 256, 256, 1e-5, eps=0.05, beta=0.5, alpha=1e-3, precision="fp64")
    plan = _pint.Plan(p)
    assert plan.work_bytes > (64 << 20)
    rep = _pint.Report()
    rep.struct_size = ct.sizeof(_pint.Report)
    u0 = torch.zeros((256, 256), dtype=torch.float64, device=dev())
    U = torch.zeros((256, 256, 256), dtype=torch.float64, device=dev())
    rc = lib.dll.pint_solve_noalloc(plan.h, u0.data_ptr(), U.data_ptr(), None, ct.byref(rep))
    assert rc == _pint.PINT_ENOMEM
    assert b"static workspace" in lib.dll.pint_plan_last_error(plan.h)
    q = _pint.make_problem("linear_ch", 2, 32, 16, 1e-5, eps=0.05, beta=0.5, alpha=1e-3, precision="fp64",
                           flags=_pint.FLAG_SOLVE_GRAPH)
    plan2 = _pint.Plan(q)
    assert lib.dll.pint_solve_noalloc(plan2.h, u0.data_ptr(), U.data_ptr(), None, ct.byref(rep)) == _pint.PINT_EINVAL
