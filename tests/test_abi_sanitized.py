"""The host interface tests (test_abi_host.py, test_equation_frontend.py)
again, in a child process, with
the host runtime built under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; device code is not instrumented).  Needs the kernel objects of the
regular build."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_interface_under_asan_and_ubsan():
    from paper_2405_02410_amd import build_hostsan as hs
    if hs.kernel_objects() is None:
        pytest.skip("kernel objects of the regular build are missing")
    hs.build()
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py"),
                        os.path.join(ROOT, "tests", "test_equation_frontend.py")],
                       cwd=ROOT, env=hs.runtime_env(), capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
