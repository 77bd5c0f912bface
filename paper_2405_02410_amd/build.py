"""Build libpss.so for gfx950 in the package directory.

The kernel source is compiled once per supported line length (8 .. 4096),
once for the fused batch kernels and once for the shared utilities, in
parallel, then linked with the host runtime.
Run as a script or call build(); both always recompile.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpss.so")
LENGTHS = (8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096)
ARCH = os.environ.get("PSS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only within one source expression, so a device
    # function rounds the same wherever it is inlined: the batched, fused and
    # LDS-resident kernels then give bit for bit the per-lattice results
    "-ffp-contract=on",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; install ROCm or set HIPCC")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build(jobs=None, verbose=False):
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    src = os.path.join(CSRC, "pss_kernels.hip")
    cmds = []
    objs = []
    for L in LENGTHS:
        o = os.path.join(BUILD, f"kern_L{L}.o")
        cmds.append([hipcc, *HIPCC_FLAGS, f"-DPSS_LINE_LEN={L}", "-c", src, "-o", o])
        objs.append(o)
    o = os.path.join(BUILD, "kern_common.o")
    cmds.append([hipcc, *HIPCC_FLAGS, "-DPSS_COMMON", "-c", src, "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "kern_batch.o")
    cmds.append([hipcc, *HIPCC_FLAGS, "-DPSS_BATCH", "-c", src, "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "noalloc.o")
    cmds.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "pss_noalloc.hip"), "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "runtime.o")
    cmds.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "pss_runtime.cpp"), "-o", o])
    objs.append(o)
    o = os.path.join(BUILD, "equation.o")
    cmds.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "pss_equation.cpp"), "-o", o])
    objs.append(o)
    jobs = jobs or min(16, os.cpu_count() or 4)
    # the longest compiles first: the fused batch kernels, then the longest lines
    weight = [L for L in LENGTHS] + [0, 100000, 0, 0, 0]
    order = sorted(range(len(cmds)), key=lambda i: -weight[i])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_run, cmds[i]) for i in order]
        for f in futs:
            out = f.result()
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
