"""The outer-iteration stop rule (CPU): the function the control kernel
calls each sweep (``csrc/stop_rule.hpp``), compiled for the host by hipcc into
``tests/stop_rule_driver.cpp`` and driven with synthetic sweep sequences.

The rule follows the error estimate of the WR / refinement iteration (its
update contracts by a rate rho per sweep, so the remaining error is about
rho / (1 - rho) times the last update) with the paper's stopping tolerance
(Section 5: 1e-10 relative); the FP64 residual guard keeps one sweep whose
update ratio dips from ending the loop while the residual grows.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINT_OK, PINT_ENOCONV, PINT_EDIVERGED = 0, -2, -3


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("stop_rule") / "driver")
    cmd = [hipcc, "-O1", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2304_14021_amd", "csrc"), os.path.join(HERE, "stop_rule_driver.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run(exe, sweeps, rtol=1e-10, safety=0.1, stagnate=0, max_iter=30):
    """sweeps: (upd, unrm, res, c_bar) per sweep -> [(k, status, done, est)]."""
    text = f"{rtol!r} {safety!r} {stagnate} {max_iter}\n" + "".join(
        f"{u!r} {n!r} {r!r} {c!r}\n" for u, n, r, c in sweeps)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    return [(int(k), int(s), int(d), float(e)) for k, s, d, e in rows]


def geometric(rate, n, res_rate=None):
    res_rate = rate if res_rate is None else res_rate
    return [(rate ** k, 1.0, 1e3 * res_rate ** k, 0.3) for k in range(n)]


def test_geometric_convergence_stops_when_the_estimate_is_below_tolerance(driver):
    # rho = 0.1: est_k = 0.1 / 0.9 * 0.1^k <= 0.1 * 1e-10 first at k = 11
    out = run(driver, geometric(0.1, 20))
    k, status, done, est = out[-1]
    assert (k, status, done) == (11, PINT_OK, 1)
    assert est == pytest.approx(0.1 / 0.9 * 1e-11, rel=1e-9)
    assert all(d == 0 for _, _, d, _ in out[:-1])


def test_residual_growth_blocks_the_estimate(driver):
    seq = geometric(0.1, 20)
    u, n, r, c = seq[11]
    seq[11] = (u, n, 2.0 * seq[10][2], c)  # the residual rises in the sweep that would stop
    out = run(driver, seq)
    assert out[11][2] == 0                  # not stopped there
    assert out[-1][:3] == (12, PINT_OK, 1)  # the next sweep (residual falling again) stops


def test_one_dipping_update_ratio(driver):
    # updates 1, 0.5, 0.25, then one tiny update: rho ~ 1e-11, est ~ 1e-23
    base = [(1.0, 1.0, 1e3, 0.3), (0.5, 1.0, 5e2, 0.3), (0.25, 1.0, 2.5e2, 0.3)]
    dip_rising = base + [(2.5e-12, 1.0, 3e2, 0.3), (0.125, 1.0, 1.2e2, 0.3)]
    out = run(driver, dip_rising)
    assert out[3][2] == 0 and out[3][3] < 1e-20   # the estimate alone would stop
    dip_falling = base + [(2.5e-12, 1.0, 1e2, 0.3)]
    assert run(driver, dip_falling)[-1][:3] == (3, PINT_OK, 1)


def test_tiny_relative_update_stops_regardless_of_the_residual(driver):
    out = run(driver, [(1.0, 1.0, 1.0, 0.3), (5e-14, 1.0, 2.0, 0.3)])
    assert out[-1][:3] == (1, PINT_OK, 1)


def test_divergence_and_nan(driver):
    grow = [(1.0, 1.0, 1.0, 0.3), (10.0, 1.0, 1.0, 0.3), (2e3, 1.0, 1.0, 0.3)]
    assert run(driver, grow)[-1][:3] == (2, PINT_EDIVERGED, 1)
    assert run(driver, [(1.0, 1.0, 1.0, float("nan"))])[-1][:3] == (0, PINT_EDIVERGED, 1)
    assert run(driver, [(1.0, 1.0, 1.0, 0.3), (float("inf"), 1.0, 1.0, 0.3)])[-1][:3] == (1, PINT_EDIVERGED, 1)


def test_out_of_iterations(driver):
    out = run(driver, geometric(0.9, 10), max_iter=5)
    assert out[-1][:3] == (4, PINT_ENOCONV, 1)


def test_unrefined_plateau(driver):
    seq = [(1.0, 1.0, 1.0, 0.3), (0.1, 1.0, 0.1, 0.3), (0.01, 1.0, 0.01, 0.3), (0.009, 1.0, 0.009, 0.3)]
    assert run(driver, seq, stagnate=1)[-1][:3] == (3, PINT_OK, 1)
    assert all(d == 0 for _, _, d, _ in run(driver, seq, stagnate=0))
