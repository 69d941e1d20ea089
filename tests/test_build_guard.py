"""Build-time register-budget guard (CPU only: hipcc cross-compiles gfx950).

A kernel that needs private scratch, accumulation registers or spills must be
refused when it is compiled; a kernel within budget passes, and every HIP
compile of the library build carries the guard."""
import os
import shutil

import pytest

from paper_1307_5310_amd import build as B

pytestmark = pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")),
                                reason="hipcc not available")

CLEAN = r"""
#include <hip/hip_runtime.h>
__global__ void residual_kernel_probe(const float* x, float* y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 2.0f * x[i];
}
"""

# a private array indexed by run-time values lives in scratch memory
OVER = r"""
#include <hip/hip_runtime.h>
__global__ void residual_kernel_probe(const float* x, const int* idx, float* y, int n) {
  float loc[96];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < 96; ++k) loc[k] = x[(i + k) % n];
  if (i < n) y[i] = loc[idx[i] % 96] + loc[idx[(i + 1) % n] % 96];
}
"""

# more live values than 128 VGPRs with 1024 threads per block: spills
SPILL = r"""
#include <hip/hip_runtime.h>
__global__ void __launch_bounds__(1024) residual_kernel_probe(const float* x, float* y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  float v[200];
#pragma unroll
  for (int k = 0; k < 200; ++k) v[k] = x[(i * 200 + k) % n];
  float s = 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 200; ++k) s = s * v[(k * 7 + r) % 200] + v[k];
  if (i < n) y[i] = s;
}
"""


def _compile(tmp_path, text, name):
    src = tmp_path / (name + ".hip")
    src.write_text(text)
    return B.compile_hip(str(src), str(tmp_path / (name + ".o")))


def test_clean_kernel_passes(tmp_path):
    _compile(tmp_path, CLEAN, "clean")


def test_scratch_kernel_refused(tmp_path):
    with pytest.raises(B.ResourceError) as ei:
        _compile(tmp_path, OVER, "over")
    assert "residual_kernel_probe" in str(ei.value) and "ScratchSize" in str(ei.value)


def test_spilling_kernel_refused(tmp_path):
    with pytest.raises(B.ResourceError) as ei:
        _compile(tmp_path, SPILL, "spill")
    msg = str(ei.value)
    assert "residual_kernel_probe" in msg and ("Spill" in msg or "ScratchSize" in msg or "AGPRs" in msg)


def test_parser_reads_every_counter():
    text = "\n".join([
        "k.hip:1:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     VGPRs: 61 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     AGPRs: 4 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:1:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
    ])
    u = B.parse_resource_remarks(text)
    assert u == {"_Z3fooPf": {"VGPRs": 61, "AGPRs": 4, "ScratchSize [bytes/lane]": 0, "VGPRs Spill": 0,
                              "SGPRs Spill": 0, "Dynamic Stack": "False"}}
    with pytest.raises(B.ResourceError, match="AGPRs 4"):
        B.check_resources(u)


def test_every_hip_compile_is_guarded():
    cmds, objs = B.commands()
    hip = [c for c in cmds if "hip" in c]
    assert len(hip) == len(B.HIP_SOURCES) + len(B.SLICES)
    for c in hip:
        assert B.GUARD_FLAG in c, c


def _sym(real, a, q, mode, aff, diss, var):
    return "_ZN4stdg15residual_kernelI%sLi%dELi%dELi%dELb%dELb%dELi%dEEEvNS_7KParamsIT_EE" % (
        "f" if real == "float" else "d", a, q, mode, aff, diss, var)


def test_register_bound_policy():
    scratch = {"AGPRs": 0, "ScratchSize [bytes/lane]": 64, "VGPRs Spill": 10, "SGPRs Spill": 0}
    agpr = {"AGPRs": 12, "ScratchSize [bytes/lane]": 0, "VGPRs Spill": 0, "SGPRs Spill": 0}
    lanes = {"AGPRs": 0, "ScratchSize [bytes/lane]": 0, "VGPRs Spill": 0, "SGPRs Spill": 40}
    # the FP32 fast path: nothing may spill
    for cnt in (scratch, agpr):
        with pytest.raises(B.ResourceError):
            B.check_resources({_sym("float", 7, 4, 0, 1, 0, 0): cnt})
    # scalar spills into vector lanes are allowed everywhere
    B.check_resources({_sym("float", 7, 4, 0, 1, 0, 0): lanes})
    # FP32 trilinear p = 8, q >= 3 is register-bound: scratch yes, AGPRs never
    B.check_resources({_sym("float", 9, 3, 0, 0, 0, 0): scratch})
    with pytest.raises(B.ResourceError, match="AGPRs"):
        B.check_resources({_sym("float", 9, 3, 0, 0, 0, 0): agpr})
    with pytest.raises(B.ResourceError):
        B.check_resources({_sym("float", 9, 2, 0, 0, 0, 0): scratch})
    # FP64 trilinear from (a, q) = (6, 3): AGPRs and scratch; below it neither
    B.check_resources({_sym("double", 6, 3, 1, 0, 0, 0): agpr})
    B.check_resources({_sym("double", 6, 3, 1, 0, 0, 0): scratch})
    with pytest.raises(B.ResourceError):
        B.check_resources({_sym("double", 6, 2, 1, 0, 0, 0): agpr})
    # every kernel outside the residual instantiations is strict
    with pytest.raises(B.ResourceError):
        B.check_resources({"_ZN4stdg12_GLOBAL__N_112pass2_kernelIdddLi16EEEv": scratch})


def test_register_bound_policy_batched_applies():
    scratch = {"AGPRs": 0, "ScratchSize [bytes/lane]": 64, "VGPRs Spill": 10, "SGPRs Spill": 0}
    # the batched apply is an affine operator-mode kernel: FP64 a = 9, q >= 3 may spill, FP32 never
    B.check_resources({"_ZN4stdg21residual_batch_kernelIdLi9ELi4EEEvNS_12BatchKParamsIT_EE": scratch})
    for name in ("_ZN4stdg21residual_batch_kernelIfLi9ELi4EEEvNS_12BatchKParamsIT_EE",
                 "_ZN4stdg21residual_batch_kernelIdLi5ELi3EEEvNS_12BatchKParamsIT_EE"):
        with pytest.raises(B.ResourceError):
            B.check_resources({name: scratch})
