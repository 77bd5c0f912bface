"""Build a host-sanitizer variant of libpss.so for the CPU interface tests.

The host runtime (pss_runtime.cpp: contexts, validation, plan compilation,
graphs, batches, tapes; pss_equation.cpp: the equation front end) is compiled with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and linked with the kernel objects of the regular
build (device code is not instrumented).  The result goes to
_build/libpss_hostsan.so; load it by setting PSS_LIB to that path and
preloading the sanitizer runtimes (runtime_env() gives the environment).
"""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(BUILD, "libpss_hostsan.so")
KERNEL_OBJECTS = [f"kern_L{L}.o" for L in (8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096)] + \
                 ["kern_common.o", "kern_batch.o", "noalloc.o"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def kernel_objects():
    """The regular build's kernel objects, or None if one is missing."""
    paths = [os.path.join(BUILD, o) for o in KERNEL_OBJECTS]
    return paths if all(os.path.exists(p) for p in paths) else None


def build():
    objs = kernel_objects()
    if objs is None:
        raise RuntimeError("kernel objects missing: run paper_2405_02410_amd.build first")
    host = []
    for src in ("pss_runtime.cpp", "pss_equation.cpp"):
        o = os.path.join(BUILD, src.replace(".cpp", "_hostsan.o"))
        compile_cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", *SAN, "-D__HIP_PLATFORM_AMD__",
                       "-I/opt/rocm/include", "-c", os.path.join(CSRC, src), "-o", o]
        subprocess.run(compile_cmd, check=True)
        host.append(o)
    link_cmd = ["g++", "-shared", *SAN, "-o", OUT + ".tmp", *host, *objs,
                "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(link_cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


def runtime_env():
    """Environment that loads the sanitized library into a plain Python."""
    libs = [subprocess.run(["g++", f"-print-file-name={n}"], capture_output=True, text=True,
                           check=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    env = dict(os.environ)
    env.update({"PSS_LIB": OUT, "LD_PRELOAD": " ".join(libs),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    return env


if __name__ == "__main__":
    print(build())
