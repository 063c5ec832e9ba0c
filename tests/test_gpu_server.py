"""The serving loop (pint_server_*) on the GPU.

A served request runs exactly the kernels of a standalone solve of the same
problem, only on a slot's stream and (after its first outer iteration) as a
replay of that slot's captured graph, so every served result must equal the
standalone result bit for bit, whatever else is in flight.  The standalone
solve itself is held to the oracle elsewhere; here a sample of the served
results is also compared with the sequential oracle directly.
"""
import ctypes as ct
import dataclasses

import numpy as np
import pytest

from oracle import stepper
from paper_2304_14021_amd import PintError, Server, Solver
from paper_2304_14021_amd import _pint
from workloads import Problem, request_u0, served_stream
from tests._gpu import dev, host, say, to_dev

pytestmark = pytest.mark.gpu
PRECS = ("mixed", "fp64", "fp32")


def _stream(n, seed=4):
    return served_stream(n_requests=n, seed=seed, grids=(16, 32, 64), nts=(16, 32, 64))


def _solo(p, u0, prec):
    s = Solver.for_problem(p, precision=prec, device=dev())
    U, rep = s.solve(to_dev(u0))
    return host(U), rep


def _serve(reqs, pool_bytes=1 << 30, max_active=4, graphs=True):
    out = []
    with Server(pool_bytes, max_active=max_active, graphs=graphs, device=dev()) as srv:
        tickets = [srv.submit(r.problem, request_u0(r), precision=PRECS[i % 3]) for i, r in enumerate(reqs)]
        for t in tickets:
            out.append(srv.wait(t, timeout_ms=120000))
        stats = srv.stats()
    return out, stats


@pytest.mark.parametrize("graphs", [True, False])
def test_served_equals_standalone_bitwise(graphs):
    reqs = _stream(12)
    say(f"server graphs={graphs}: {[(r.problem.op[:3], r.problem.n, r.problem.nt) for r in reqs]}")
    res, st = _serve(reqs, graphs=graphs)
    for i, (r, (U, rep)) in enumerate(zip(reqs, res)):
        prec = PRECS[i % 3]
        ref, rrep = _solo(r.problem, request_u0(r), prec)
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, ref), f"request {i} ({prec}) differs from the standalone solve"
    say(f"  stats {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["queued"] == 0 and st["active"] == 0
    assert st["pool_in_use"] == 0 and 0 < st["pool_peak"] <= st["pool_bytes"]
    assert st["dof_completed"] == sum(r.problem.dof for r in reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    if graphs:
        assert st["graphs_captured"] >= 1 and st["graph_launches"] >= 1
    else:
        assert st["graphs_captured"] == 0 and st["graph_launches"] == 0


def test_served_against_oracle():
    reqs = _stream(6, seed=7)
    res, _ = _serve(reqs, max_active=3)
    for i, (r, (U, rep)) in enumerate(zip(reqs, res)):
        err = stepper.rel_err(U, stepper.sequential(r.problem, request_u0(r)))
        say(f"  request {i} {r.problem.op} n{r.problem.n} nt{r.problem.nt} {PRECS[i % 3]}: "
            f"it {rep['iterations']} err {err:.2e}")
        assert err <= 1e-10


@pytest.mark.skip(reason="a GPU memory fault was observed in this test's run (illegal address at the "
                         "standalone solve after the served requests) while executable graphs were "
                         "re-targeted with hipGraphExecUpdate; its cause was not shown, that path has been "
                         "removed from the server, and this case stays off the GPU")
def test_graph_reuse_within_a_shape_class():
    # one slot, several requests of one shape class with different
    # coefficients: one capture, then executable-graph updates (path removed)
    base = Problem(op="linear_ch", dim=2, n=32, nt=32, dt=1e-5, eps=0.05, beta=0.3, alpha=1e-3)
    ps = [dataclasses.replace(base, eps=e) for e in (0.03, 0.05, 0.07)]
    rng = np.random.default_rng(3)
    u0s = [rng.uniform(-0.05, 0.05, base.slice_shape) for _ in ps]
    with Server(1 << 28, max_active=1, device=dev()) as srv:
        ts = [srv.submit(p, u, precision="fp64") for p, u in zip(ps, u0s)]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    say(f"  stats {st}")
    assert st["graphs_captured"] + st["graph_updates"] == len(ps)
    assert st["graphs_captured"] >= 1
    for p, u0, (U, rep) in zip(ps, u0s, res):
        ref, _ = _solo(p, u0, "fp64")
        assert np.array_equal(U, ref)


def _footprint(p, prec):
    with Server(1 << 28, max_active=1, device=dev()) as srv:
        srv.wait(srv.submit(p, np.zeros(p.slice_shape), precision=prec))
        return srv.stats()["pool_peak"]


def test_admission_by_pool_memory():
    p = Problem(op="biharmonic", dim=2, n=64, nt=64, dt=1e-5, alpha=1e-3)
    fp = _footprint(p, "mixed")
    say(f"  footprint of one 64^2 x 64 request: {fp} bytes")
    rng = np.random.default_rng(5)
    u0s = [rng.uniform(-0.05, 0.05, p.slice_shape) for _ in range(4)]
    # room for one request only, though four slots are free
    with Server(fp + 4096, max_active=4, device=dev()) as srv:
        ts = [srv.submit(p, u, precision="mixed") for u in u0s]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    assert st["completed"] == 4 and st["pool_peak"] == fp
    for u0, (U, _) in zip(u0s, res):
        ref, _ = _solo(p, u0, "mixed")
        assert np.array_equal(U, ref)


def test_submit_errors():
    with Server(1 << 20, max_active=2, device=dev()) as srv:
        big = Problem(op="biharmonic", dim=2, n=128, nt=128, dt=1e-5, alpha=1e-3)
        with pytest.raises(PintError) as e:
            srv.submit(big, np.zeros(big.slice_shape))
        assert e.value.code == _pint.PINT_ENOMEM
        bad = _pint.make_problem("biharmonic", 2, 24, 16, 1e-5)  # grid not a power of two
        with pytest.raises(PintError) as e:
            srv.submit(bad, np.zeros(24 * 24))
        assert e.value.code == _pint.PINT_EINVAL
        with pytest.raises(PintError) as e:
            srv.wait(12345)
        assert e.value.code == _pint.PINT_ENOTFOUND
        with pytest.raises(ValueError):
            srv.submit(Problem(op="biharmonic", dim=2, n=16, nt=16, dt=1e-5), np.zeros(15))
        st = srv.stats()
    assert st["submitted"] == 0 and st["failed"] == 0
    with Server(1 << 26, max_active=2, device=dev(), host_pool_bytes=1 << 16) as srv2:
        mid = Problem(op="biharmonic", dim=2, n=32, nt=16, dt=1e-5, alpha=1e-3)  # 128 KiB result
        with pytest.raises(PintError) as e:
            srv2.submit(mid, np.zeros(mid.slice_shape))
        assert e.value.code == _pint.PINT_ENOMEM


def test_cancel_and_timeout():
    head = Problem(op="linear_ch", dim=2, n=128, nt=256, dt=1e-5, eps=0.05, beta=0.3, alpha=1e-3)
    tail = Problem(op="biharmonic", dim=2, n=32, nt=32, dt=1e-5, alpha=1e-3)
    rng = np.random.default_rng(6)
    u0h = rng.uniform(-0.05, 0.05, head.slice_shape)
    u0t = rng.uniform(-0.05, 0.05, tail.slice_shape)
    with Server(1 << 30, max_active=1, device=dev()) as srv:
        t1 = srv.submit(head, u0h, precision="fp64")
        t2 = srv.submit(tail, u0t, precision="fp64")
        t3 = srv.submit(tail, u0t, precision="fp64")
        srv.cancel(t2)
        with pytest.raises(PintError) as e:   # t3 queues behind t1 on the single slot
            srv.wait(t3, timeout_ms=0)
        assert e.value.code == _pint.PINT_ETIMEDOUT
        U1, r1 = srv.wait(t1)
        _, r2 = srv.wait(t2, raise_on_error=False)
        U3, r3 = srv.wait(t3)
        st = srv.stats()
    assert r1["status"] == 0 and r2["status"] == _pint.PINT_ECANCELED and r3["status"] == 0
    assert st["completed"] == 2 and st["cancelled"] == 1
    assert np.array_equal(U3, _solo(tail, u0t, "fp64")[0])
    assert np.array_equal(U1, _solo(head, u0h, "fp64")[0])


def test_device_resident_requests():
    # device-resident and host requests mixed in one server: each device result
    # equals the standalone solve bit for bit, and only tables + workspace come
    # from the pool
    import torch
    reqs = _stream(8, seed=9)
    with Server(1 << 30, max_active=4, device=dev()) as srv:
        bufs, ts = [], []
        for i, r in enumerate(reqs):
            u0 = request_u0(r)
            if i % 2 == 0:
                d0 = to_dev(u0)
                dU = torch.full(r.problem.shape, float("nan"), dtype=torch.float64, device=dev())
                ts.append(srv.submit_device(r.problem, d0, dU, precision=PRECS[i % 3]))
                bufs.append(dU)
            else:
                ts.append(srv.submit(r.problem, u0, precision=PRECS[i % 3]))
                bufs.append(None)
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
        with pytest.raises(PintError) as e:   # overlapping input and output
            big = torch.zeros((16 + 1) * 16 * 16, dtype=torch.float64, device=dev())
            p = Problem(op="biharmonic", dim=2, n=16, nt=16, dt=1e-5)
            srv._check(srv.lib.dll.pint_server_submit_device(
                srv.h, ct.byref(srv._struct(p, "fp64", 1e-10, 30)), big.data_ptr() + 8 * 16 * 16,
                big.data_ptr(), ct.byref(ct.c_uint64())), srv.h)
        assert e.value.code == _pint.PINT_EINVAL
    assert st["completed"] == len(reqs)
    for i, (r, (U, rep)) in enumerate(zip(reqs, res)):
        ref, _ = _solo(r.problem, request_u0(r), PRECS[i % 3])
        got = host(U) if bufs[i] is not None else U
        if bufs[i] is not None:
            assert U is bufs[i]
        assert rep["status"] == 0 and np.array_equal(got, ref), f"request {i}"


def test_host_results_wait_in_pinned_pool_until_collected():
    # a finished host-buffer request frees its device block and keeps U in the
    # pinned result pool until wait copies it out
    import time
    p = Problem(op="biharmonic", dim=2, n=32, nt=32, dt=1e-5, alpha=1e-3)
    u0 = np.random.default_rng(12).uniform(-0.05, 0.05, p.slice_shape)
    with Server(1 << 26, max_active=2, device=dev(), host_pool_bytes=1 << 24) as srv:
        t = srv.submit(p, u0, precision="fp64")
        t_end = time.time() + 60
        while srv.stats()["completed"] < 1 and time.time() < t_end:
            time.sleep(1e-3)
        st = srv.stats()
        assert st["completed"] == 1 and st["active"] == 0 and st["pool_in_use"] == 0
        assert st["host_pool_in_use"] == p.dof * 8 and st["host_pool_bytes"] == 1 << 24
        U, rep = srv.wait(t)
        assert srv.stats()["host_pool_in_use"] == 0
    assert np.array_equal(U, _solo(p, u0, "fp64")[0])


def test_served_dense_bf16_requests():
    # requests on the dense matrix-core time path (BF16 split), replayed from
    # captured graphs, equal their standalone solves bit for bit
    base = Problem(op="linear_ch", dim=2, n=64, nt=64, dt=1e-5, eps=0.05, beta=0.3, alpha=1e-2)
    ps = [dataclasses.replace(base, eps=e) for e in (0.04, 0.06)]
    rng = np.random.default_rng(17)
    u0s = [rng.uniform(-0.05, 0.05, base.slice_shape) for _ in ps]
    with Server(1 << 28, max_active=2, device=dev()) as srv:
        ts = [srv.submit(p, u, precision="bf16x3") for p, u in zip(ps, u0s)]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    assert st["completed"] == 2 and st["graph_launches"] >= 1
    for p, u0, (U, rep) in zip(ps, u0s, res):
        ref, rrep = _solo(p, u0, "bf16x3")
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, ref)
        assert stepper.rel_err(U, stepper.sequential(p, u0)) <= 1e-10


def test_served_fp64_small_alpha_two_steps():
    # the benchmark's served configuration: FP64 requests at alpha = 1e-6 take
    # two outer iterations each and meet the 1e-10 bar against the oracle
    reqs = served_stream(n_requests=6, seed=11, grids=(64, 128), nts=(32, 64, 128))
    reqs = [dataclasses.replace(r, problem=dataclasses.replace(r.problem, alpha=1e-6)) for r in reqs]
    with Server(1 << 30, max_active=3, device=dev()) as srv:
        res = [srv.wait(t, timeout_ms=120000) for t in
               [srv.submit(r.problem, request_u0(r), precision="fp64") for r in reqs]]
    for i, (r, (U, rep)) in enumerate(zip(reqs, res)):
        err = stepper.rel_err(U, stepper.sequential(r.problem, request_u0(r)))
        say(f"  request {i} {r.problem.op} n{r.problem.n} nt{r.problem.nt} fp64 alpha 1e-6: "
            f"it {rep['iterations']} err {err:.2e}")
        assert rep["status"] == 0 and rep["iterations"] == 2 and err <= 1e-10


def test_served_dense_and_fft_requests_of_one_shape():
    # requests that differ only in their time path (dense FP32 MFMA vs FFT) and
    # coefficients, on two slots: each one is captured on its own, and every
    # result equals its standalone solve bit for bit
    shape = dict(op="linear_ch", dim=2, n=32, nt=32, dt=1e-5, beta=0.3, alpha=1e-3)
    combos = [("dense", 0.03), ("fft", 0.05), ("dense", 0.07), ("fft", 0.04)]
    rng = np.random.default_rng(23)
    u0s = [rng.uniform(-0.05, 0.05, (32, 32)) for _ in combos]
    structs = [_pint.make_problem(shape["op"], 2, 32, 32, 1e-5, eps=e, beta=0.3, alpha=1e-3, precision="mixed",
                                  time_path=tp) for tp, e in combos]
    say(f"served dense/fft mix: {combos}")
    with Server(1 << 28, max_active=2, device=dev()) as srv:
        ts = [srv.submit(q, u) for q, u in zip(structs, u0s)]
        res = [srv.wait(t) for t in ts]
        st = srv.stats()
    say(f"  stats {st}")
    assert st["completed"] == len(combos) and st["graph_updates"] == 0
    assert st["graphs_captured"] == len(combos)
    for (tp, e), u0, (U, rep) in zip(combos, u0s, res):
        s = Solver(shape["op"], 2, 32, 32, 1e-5, eps=e, beta=0.3, alpha=1e-3, precision="mixed", time_path=tp,
                   device=dev())
        Ud, rrep = s.solve(to_dev(u0))
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, host(Ud)), f"{tp} eps {e}"


def test_served_panel_layout_requests():
    # 2D requests with N_t >= 512 keep their time solve's spectral array in
    # line-wide panels (a second spectral buffer in the request's pool block):
    # served beside plain-layout ones, each equals its standalone solve bit for
    # bit and the sequential oracle within 1e-10
    probs = [Problem(op="ch", dim=2, n=16, nt=512, dt=1e-6, eps=0.05, alpha=1e-3),
             Problem(op="biharmonic", dim=2, n=8, nt=1024, dt=1e-5, theta=0.5, alpha=1e-3),
             Problem(op="linear_ch", dim=2, n=16, nt=64, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3)]
    rng = np.random.default_rng(29)
    u0s = [rng.uniform(-0.3, 0.3, p.slice_shape) for p in probs]
    jobs = [(p, u, prec) for p, u in zip(probs, u0s) for prec in PRECS]
    say(f"served panel-layout requests: {[(p.op[:3], p.n, p.nt, prec) for p, _, prec in jobs]}")
    with Server(1 << 28, max_active=3, device=dev()) as srv:
        ts = [srv.submit(p, u, precision=prec) for p, u, prec in jobs]
        res = [srv.wait(t, timeout_ms=120000) for t in ts]
    for (p, u0, prec), (U, rep) in zip(jobs, res):
        ref, rrep = _solo(p, u0, prec)
        assert rep["status"] == 0 and rep["iterations"] == rrep["iterations"]
        assert np.array_equal(U, ref), f"{p.op} nt {p.nt} {prec}"
        err = stepper.rel_err(U, stepper.sequential(p, u0))
        assert err <= 1e-10, (p.op, p.nt, prec, err)
