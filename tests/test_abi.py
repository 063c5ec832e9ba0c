"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, the ctypes structures match the C layout, and argument
validation rejects bad problems before any device work."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np

import pytest

from paper_2304_14021_amd import _pint

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pint.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pint_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _pint.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib.dll, n), n
    assert set(names) == set(_pint.EXPORTS)
    assert b"gfx950" in lib.dll.pint_version()


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "pint.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pint_problem), sizeof(pint_report),'
                   ' offsetof(pint_problem, flags), offsetof(pint_report, ms_total), offsetof(pint_problem, rtol),'
                   ' sizeof(pint_server_config), sizeof(pint_server_statistics),'
                   ' offsetof(pint_server_statistics, worker_host_seconds));'
                   'printf("%zu %zu\\n", offsetof(pint_report, mass_drift), offsetof(pint_report, energy_monotone));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ct.sizeof(_pint.Problem), ct.sizeof(_pint.Report), _pint.Problem.flags.offset,
            _pint.Report.ms_total.offset, _pint.Problem.rtol.offset, ct.sizeof(_pint.ServerConfig),
            ct.sizeof(_pint.ServerStats), _pint.ServerStats.worker_host_seconds.offset,
            _pint.Report.mass_drift.offset, _pint.Report.energy_monotone.offset]
    assert [int(x) for x in got] == want


@pytest.mark.parametrize("kw,frag", [
    (dict(n=100), "power of two"),
    (dict(n=4), "power of two"),
    (dict(nt=3), "power of two"),
    (dict(nt=2048), "power of two"),
    (dict(dt=0.0), "dt"),
    (dict(theta=0.7), "theta"),
    (dict(alpha=1.5), "alpha"),
    (dict(alpha=0.9), "admissible"),
    (dict(eps=0.0), "eps"),
    (dict(max_iter=100), "max_iter"),
])
def test_validation_rejects_bad_problems(kw, frag):
    args = dict(op="linear_ch", dim=2, n=32, nt=16, dt=1e-5, eps=0.05, beta=0.5, alpha=1e-3)
    args.update(kw)
    if kw.get("alpha") == 0.9:
        # alpha * R^Nt >= 1/2 for a strongly spinodal problem
        args.update(dt=1e-3, nt=64, beta=0.57, eps=0.02)
    p = _pint.make_problem(**args)
    with pytest.raises(_pint.PintError) as ei:
        _pint.Plan(p)
    assert ei.value.code == _pint.PINT_EINVAL
    assert frag in str(ei.value)


def test_status_strings():
    lib = _pint.lib()
    for code in range(-8, 1):
        assert lib.dll.pint_status_string(code).startswith(b"PINT_")


@pytest.mark.parametrize("kw,frag", [
    (dict(dts=np.full(32, 1e-5)), "pairwise distinct"),
    (dict(dts=np.r_[-1e-5, 1e-5 * 1.1 ** np.arange(1, 32)]), "> 0"),
    (dict(op="ch_eyre"), "Eyre"),
    (dict(precision="bf16"), "precision"),
    (dict(time_path="fft"), "FFT"),
    (dict(nt=16, dts=1e-6 * 1.2 ** np.arange(16)), "nt >= 32"),
])
def test_validation_rejects_bad_nonuniform_steps(kw, frag):
    # checked before any device work (no GPU needed)
    args = dict(op="linear_ch", dim=2, n=32, nt=32, dt=0.0, eps=0.05, beta=0.5, precision="mixed",
                dts=1e-6 * 1.2 ** np.arange(32))
    args.update(kw)
    p = _pint.make_problem(**args)
    with pytest.raises(_pint.PintError) as ei:
        _pint.Plan(p)
    assert ei.value.code == _pint.PINT_EINVAL
    assert frag in str(ei.value)
