"""The debug and tuning-cache environment switches, on the GPU, through the C
interface.

PSS_DEBUG_SYNC (read when a lattice is created) makes pss_step enqueue the
step's kernels one by one, synchronise and check after each, and fill the
workspaces with NaN when they are allocated.  Checks: every kind of lattice
(1D, 2D, 3D, mixed-radix sizes, Model H with intermediates, frames) ends
bitwise where the graph path ends, so no kernel reads a workspace before
writing it and the eager path keys the noise by the same steps; a NaN put
into the state is reported by pss_step itself, naming the kernel and the
step.

PSS_TUNE_CACHE names a file that keeps pss_autotune's choices: an autotune in
one process appends one line; a second process with the same lattice takes
the geometry and the recorded time from it, to the last bit, and appends
nothing; lines that do not parse are skipped.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import PssError  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _model_b(n, seed=4):
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    f, _ = pss.model_b(lat, D=0.02)
    lat.init_uniform(f, -0.2, 0.2)
    return lat, [f]


def _model_h(n, seed=6):
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    ids, grads = pss.model_h(lat, a=-1.0, b=1.0, k=1.0, M=1.0, eta=0.5, D=0.01)
    lat.init_uniform(ids[0], -0.4, 0.4)
    return lat, list(ids) + list(grads)


def _framed(n, seed=5):
    lat, ids = _model_b(n, seed)
    sites = [y * n[0] + x for y in range(n[1]) for x in range(3)]
    lat.frame(ids[0], sites, [0.25] * len(sites))
    return lat, ids


CASES = [
    ("2d model b", lambda: _model_b((256, 128)), 40),
    ("1d model b", lambda: _model_b((512,)), 60),
    ("1d mixed", lambda: _model_b((96,)), 60),
    ("3d model b", lambda: _model_b((32, 16, 32)), 20),
    ("2d mixed", lambda: _model_b((96, 64)), 30),
    ("3d mixed", lambda: _model_b((24, 16, 12)), 15),
    ("2d model h", lambda: _model_h((128, 64)), 30),
    ("3d model h", lambda: _model_h((16, 16, 16)), 15),
    ("2d frames", lambda: _framed((128, 64)), 30),
]


@pytest.mark.parametrize("name,build,steps", CASES, ids=[c[0] for c in CASES])
def test_debug_mode_is_bitwise_the_graph_path(monkeypatch, name, build, steps):
    print(f"debug sync {name} steps={steps}", flush=True)
    monkeypatch.delenv("PSS_DEBUG_SYNC", raising=False)
    ref, ids = build()
    monkeypatch.setenv("PSS_DEBUG_SYNC", "1")
    dbg, _ = build()
    monkeypatch.delenv("PSS_DEBUG_SYNC")
    ref.step(steps)
    dbg.step(steps // 3)
    dbg.step(steps - steps // 3)
    assert dbg.step_index == ref.step_index == steps
    for f in ids:
        a, b = dbg.download(f), ref.download(f)
        assert np.all(np.isfinite(a)), f
        assert np.array_equal(a, b), f


def test_debug_mode_names_the_kernel_and_step_of_a_nan(monkeypatch):
    monkeypatch.setenv("PSS_DEBUG_SYNC", "1")
    lat, (f,) = _model_b((128, 64))
    lat.step(5)
    x = lat.download(f)
    x[3, 7] = np.nan
    lat.upload(f, x)
    with pytest.raises(PssError) as e:
        lat.step(10)
    assert e.value.name == "PSS_E_NONFINITE"
    assert "update_kernel" in str(e.value) and "step 5" in str(e.value), str(e.value)
    assert lat.step_index == 5


_CHILD = """
import json, sys
sys.path.insert(0, {root!r})
import paper_2405_02410_amd as pss
lat = pss.Lattice((256, 128), dt=0.01, seed=1)
pss.model_b(lat)
us = lat.autotune(reps=10)
print(json.dumps({{"us": us, "geo": lat.geometry()}}))
"""


def _child(path):
    env = dict(os.environ, PSS_TUNE_CACHE=str(path))
    env.pop("PSS_DEBUG_SYNC", None)
    r = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=150)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tuning_cache_file_across_processes(tmp_path):
    path = tmp_path / "tune.txt"
    path.write_text("not a cache line\nv1/x/2x256x128 -1 tc=3\n")
    first = _child(path)
    lines = path.read_text().splitlines()
    assert len(lines) == 3
    key, us, *kv = lines[-1].split()
    assert key.startswith("v1/gfx950") and "2x256x128" in key
    assert float(us) == first["us"]
    second = _child(path)
    assert second == first
    assert len(path.read_text().splitlines()) == 3
