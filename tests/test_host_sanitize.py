"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the mesh
builder (faces, orientations, split-face and geometry checks, metric, groups)
and the 1D tables, compiled for the host only with g++ into a harness
(tests/host/mesh_sanitize.cpp) that runs valid meshes in every orientation and
invalid inputs that must be refused.  No device code, no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIP_INCLUDE = "/opt/rocm/include"
HIP_LIB = "/opt/rocm/lib"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INCLUDE),
                    reason="needs g++ and the HIP headers")
def test_mesh_builder_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "mesh_sanitize")
    csrc = os.path.join(ROOT, "paper_1307_5310_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE,
           "-o", exe, os.path.join(HERE, "host", "mesh_sanitize.cpp"), os.path.join(csrc, "mesh.cpp"),
           os.path.join(csrc, "tables.cpp"), "-L" + HIP_LIB, "-lamdhip64", "-Wl,-rpath," + HIP_LIB]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "all cases as expected" in r.stdout
