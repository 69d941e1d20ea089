"""The library's time tables of local time steps (Section 2.2; S_h of
Section 4.1, eq. bilinearform:S), built on the host from closed forms and
Gauss rules (tables.cpp), against the oracle's tables, which integrate the
projected sub-interval test functions against the flattened trial functions
by composite quadrature; and D_h's own part (the own trial against the
projected test function).  A g++ build of tables.cpp with a small harness
(tests/host/lt_tables.cpp); no device code, no GPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import basis

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIP_INCLUDE = "/opt/rocm/include"
HIP_LIB = "/opt/rocm/lib"


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(HIP_INCLUDE):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("lt") / "lt_tables")
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE, "-o", exe,
           os.path.join(HERE, "host", "lt_tables.cpp"), os.path.join(ROOT, "paper_1307_5310_amd", "csrc", "tables.cpp"),
           "-L" + HIP_LIB, "-lamdhip64", "-Wl,-rpath," + HIP_LIB]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    return exe


def _tables(exe, q, n, qk, nk):
    out = subprocess.run([exe, str(q), str(n), str(qk), str(nk)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0
    lines = out.stdout.split("\n")
    D = np.array(lines[0].split()[3:], float).reshape(n * q, 1 + n * q)
    N = np.array(lines[1].split()[3:], float).reshape(n * q, 1 + n * q)
    C = np.array(lines[2].split()[5:], float).reshape(n * q, 1 + nk * qk)
    Pt = np.array(lines[3].split()[5:], float).reshape(n * q, 1 + n * q)
    return D, N, C, Pt


@pytest.mark.parametrize("q,n", [(1, 1), (1, 2), (2, 4), (3, 8), (6, 4), (4, 2)])
def test_tables_match_the_oracle(harness, q, n):
    for qk in (1, 2, 3, 5):
        for nk in (1, 2, 4, 8):
            if nk * qk > 24:
                continue
            D, N, C, Pt = _tables(harness, q, n, qk, nk)
            assert np.abs(D - basis.subinterval_time_table(q, n, q, n, deriv=True)).max() < 1e-13
            assert np.abs(N - basis.subinterval_time_table(q, n, q, n)).max() < 1e-13
            Co = basis.subinterval_time_table(q, n, qk, nk, proj=(min(q, qk), min(n, nk)))
            assert np.abs(C - Co).max() < 1e-13, (q, n, qk, nk)
            Po = basis.subinterval_time_table(q, n, q, n, proj=(min(q, qk), min(n, nk)))
            assert np.abs(Pt - Po).max() < 1e-13, (q, n, qk, nk)
