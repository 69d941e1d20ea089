"""Build libstdg.so in-tree for gfx950 with hipcc.

Every call recompiles every source (objects go to ``_build/`` next to this
file; the library is ``libstdg.so`` in this package directory).  The residual
kernels are compiled once per (precision, a = p + 1, affine or trilinear, with or
without the dissipative face terms) slice so the slices build in parallel.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstdg.so")

HOST_SOURCES = ["api.cpp", "mesh.cpp", "tables.cpp", "solver.cpp", "serve.cpp"]
HIP_SOURCES = ["residual.hip", "blas.hip", "krylov.hip", "load.hip", "dualnorm.hip"]
# (precision, a, affine, dissipative): the dissipative variants exist for affine elements only
SLICES = [(real, a, aff, 0) for real in ("float", "double") for a in range(2, 10) for aff in (1, 0)] + \
         [(real, a, 1, 1) for real in ("float", "double") for a in range(2, 10)]

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I" + os.path.join(HERE, "..", "include")]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(jobs=None, verbose=False):
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for src in HOST_SOURCES + HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([hipcc] + COMMON + lang + ["-c", path, "-o", obj])
        objs.append(obj)
    for real, a, aff, diss in SLICES:
        obj = os.path.join(BUILD, "residual_%s_a%d_%s%s.o" % (real, a, "aff" if aff else "tri", "_diss" if diss else ""))
        cmds.append([hipcc] + COMMON + ["-x", "hip", "-DSTDG_REAL=%s" % real, "-DSTDG_A=%d" % a,
                                        "-DSTDG_AFF=%d" % aff, "-DSTDG_DISS=%d" % diss,
                                        "-c", os.path.join(CSRC, "residual_inst.hip"), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
