"""The launch-geometry autotuner (pss_autotune): it picks a valid geometry, is
no slower than the default in its own timing, keeps forced keys, caches per
shape, and the tuned lattice stays on the oracle."""

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402


def _model_b(n, seed=3):
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    f, _ = pss.model_b(lat)
    return lat, f


def _step_time(lat, reps=50):
    return sum(lat.time_kernel(w, reps)[0] for w in range(lat.kernels_per_step())) * 1e3


@pytest.mark.parametrize("n", [(128, 128), (256, 64), (64, 64, 64)])
def test_autotuned_lattice_is_valid_fast_and_on_the_oracle(n):
    lat, f = _model_b(n)
    us = lat.autotune(reps=20)
    assert np.isfinite(us) and us > 0
    lat.init_uniform(f)
    g = lat.geometry()
    ref, fr = _model_b(n)
    ref.init_uniform(fr)
    lat.step(30)
    ref.step(30)
    assert np.max(np.abs(lat.download(f) - ref.download(fr))) < 1e-5
    if len(n) == 2:
        p = inputs.MODEL_B
        m = om.model_b(OLattice(n[0], n[1], 1), p["dt"], a=p["a"], b=p["b"], k=p["k"], D=0.01, seed=3)
        m.init_uniform(0, -0.1, 0.1)
        m.step(30)
        assert np.max(np.abs(lat.download(f) - m.real(0)[0])) < 2e-5
    # its own choice against the default, re-timed (lenient: timing noise)
    assert _step_time(lat) <= 1.25 * _step_time(ref), (g, ref.geometry())


def test_autotune_keeps_forced_keys_and_caches():
    a, fa = _model_b((128, 64))
    a.tune(tc=2)
    a.autotune(reps=10)
    a.init_uniform(fa)
    assert a.geometry()["tc"] == 2
    b, fb = _model_b((128, 64))
    b.tune(tc=2)
    b.autotune(reps=10)  # cache hit: same choice
    b.init_uniform(fb)
    assert b.geometry() == a.geometry()
    with pytest.raises(pss.PssError) as e:
        b.autotune()
    assert e.value.name == "PSS_E_STATE"
