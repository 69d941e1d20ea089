"""Build libstdg.so in-tree for gfx950 with hipcc.

Every call recompiles every source (objects go to ``_build/`` next to this
file; the library is ``libstdg.so`` in this package directory).  The residual
kernels are compiled once per (precision, a = p + 1, affine or trilinear, with or
without the dissipative face terms) slice so the slices build in parallel.

Resource guard: every HIP source is compiled with the compiler's kernel
resource-usage remarks, and the build fails when a kernel uses accumulation
registers (AGPRs), private scratch memory or vector register spills, except
the register-bound residual instantiations listed in REGISTER_BOUND (FP64 at
high p q, FP32 trilinear at p = 8).  On gfx950 a kernel past 256 VGPRs moves
values into AGPRs; FP32 residual kernels of that kind have given wrong
results without any error, so no FP32 kernel may use them.
"""
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libstdg.so")

HOST_SOURCES = ["api.cpp", "mesh.cpp", "tables.cpp", "solver.cpp", "serve.cpp"]
HIP_SOURCES = ["residual.hip", "blas.hip", "krylov.hip", "load.hip", "dualnorm.hip", "dissipation.hip", "hanging.hip",
               "local_time.hip"]
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


GUARD_FLAG = "-Rpass-analysis=kernel-resource-usage"
# resource counters of the remarks that must read zero
GUARD_ZERO = ("AGPRs", "ScratchSize [bytes/lane]", "VGPRs Spill")
# Register-bound residual instantiations: (precision, kind) -> {a: smallest q}
# from which the element's live state (its own block over all q + 1 levels,
# the time-contracted face traces, with trilinear elements the quadrature
# mass) no longer fits 256 VGPRs at one wave per SIMD.  These may spill, to
# scratch or (FP64 only) into AGPRs; they are correct (parity-tested) but
# slow.  Every other kernel - the FP32 path below p = 8 in particular - must
# be free of AGPRs, scratch and spills.  Scalar spills go to vector lanes
# when the scratch size is zero and are allowed everywhere.
REGISTER_BOUND = {
    ("double", "affine"): {8: 6, 9: 3},
    ("double", "diss"): {5: 6, 6: 5, 7: 5, 8: 4, 9: 2},
    ("double", "trilinear"): {2: 6, 3: 5, 4: 5, 5: 4, 6: 3, 7: 2, 8: 2, 9: 1},
    ("float", "trilinear"): {9: 3},
}
_RESID = re.compile(r"residual_kernelI([fd])Li(\d+)ELi(\d+)ELi(\d+)ELb([01])ELb([01])ELi(\d+)E")
_RESID_BATCH = re.compile(r"residual_batch_kernelI([fd])Li(\d+)ELi(\d+)E")  # affine, operator mode


class ResourceError(RuntimeError):
    """A kernel exceeds the register budget (AGPRs, scratch or spills)."""


def parse_resource_remarks(text):
    """{kernel symbol: {counter: value}} from kernel-resource-usage remarks."""
    out = {}
    cur = None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?): (\S+) \[-Rpass-analysis=kernel-resource-usage\]", line)
        if m and cur is not None:
            v = m.group(2)
            cur[m.group(1).strip()] = int(v) if v.isdigit() else v
    return out


def allowed_counters(name):
    """The guarded counters that may be nonzero for this kernel symbol."""
    m = _RESID.search(name)
    if m:
        kind = "diss" if m.group(6) == "1" else ("affine" if m.group(5) == "1" else "trilinear")
    else:
        m = _RESID_BATCH.search(name)
        if not m:
            return ()
        kind = "affine"
    real = "float" if m.group(1) == "f" else "double"
    a, q = int(m.group(2)), int(m.group(3))
    qmin = REGISTER_BOUND.get((real, kind), {}).get(a)
    if qmin is None or q < qmin:
        return ()
    return ("ScratchSize [bytes/lane]", "VGPRs Spill") + (("AGPRs",) if real == "double" else ())


def check_resources(usage, source=""):
    """Raise ResourceError naming every kernel over its budget."""
    bad = []
    for name, cnt in sorted(usage.items()):
        ok = allowed_counters(name)
        over = ["%s %s" % (k, cnt[k]) for k in GUARD_ZERO
                if k not in ok and isinstance(cnt.get(k), int) and cnt[k] != 0]
        if over:
            bad.append("%s: %s" % (name, ", ".join(over)))
    if bad:
        raise ResourceError("kernel register budget exceeded in %s:\n  " % (source or "a HIP source") +
                            "\n  ".join(bad))
    return usage


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    if GUARD_FLAG in cmd:
        usage = check_resources(parse_resource_remarks(p.stdout), cmd[cmd.index("-c") + 1])
        if not usage and "--offload-arch=gfx950" in cmd:
            src = cmd[cmd.index("-c") + 1]
            with open(src) as f:
                if "__global__" in f.read():
                    raise ResourceError("no kernel resource remarks from %s (compiler output changed?)" % src)
        # keep the output free of the remarks themselves
        return "\n".join(l for l in p.stdout.splitlines() if "kernel-resource-usage" not in l and
                         not l.lstrip().startswith(("|", "^")) and not re.match(r"\s*\d+ \|", l))
    return p.stdout


def compile_hip(src, obj, defines=()):
    """Compile one HIP source for gfx950 under the resource guard."""
    return _run([_hipcc()] + COMMON + [GUARD_FLAG, "-x", "hip"] + ["-D" + d for d in defines] +
                ["-c", src, "-o", obj])


def commands():
    """(compile commands, object files) of every source; HIP ones carry the guard."""
    hipcc = _hipcc()
    cmds = []
    objs = []
    for src in HOST_SOURCES + HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src.replace(".", "_") + ".o")
        lang = [GUARD_FLAG, "-x", "hip"] if src.endswith(".hip") else []
        cmds.append([hipcc] + COMMON + lang + ["-c", path, "-o", obj])
        objs.append(obj)
    for real, a, aff, diss in SLICES:
        obj = os.path.join(BUILD, "residual_%s_a%d_%s%s.o" % (real, a, "aff" if aff else "tri", "_diss" if diss else ""))
        cmds.append([hipcc] + COMMON + [GUARD_FLAG, "-x", "hip", "-DSTDG_REAL=%s" % real, "-DSTDG_A=%d" % a,
                                        "-DSTDG_AFF=%d" % aff, "-DSTDG_DISS=%d" % diss,
                                        "-c", os.path.join(CSRC, "residual_inst.hip"), "-o", obj])
        objs.append(obj)
    return cmds, objs


def build(jobs=None, verbose=False):
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    cmds, objs = commands()
    jobs = jobs or min(16, os.cpu_count() or 4)
    def attempt(cmd):
        try:
            return _run(cmd), None
        except RuntimeError as e:
            return None, e

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        res = list(ex.map(attempt, cmds))
    errs = [e for _, e in res if e is not None]
    if errs:
        # every failing source, the resource guard's first when it fired
        errs.sort(key=lambda e: not isinstance(e, ResourceError))
        raise type(errs[0])("\n".join(str(e) for e in errs))
    outs = [o for o, _ in res]
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
