"""The allocation-free structure-factor entry point (pss_structure_factor_noalloc)
against pss_structure_factor, through the C interface: two calls in a row on
the same GPU, the second on a smaller lattice (the shared static scratch keeps
the first call's contents and must be cleared), and the argument checks.

Both calls run the same kernels, whose shell sums are exact integer sums
(independent of the order of the atomics): counts and S_j agree bit for bit."""

import ctypes

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402


def _lattice(n, seed, steps):
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    f, _ = pss.model_b(lat)
    lat.init_uniform(f, -0.1, 0.1)
    lat.step(steps)
    lat.sync()
    return lat


def _raw_noalloc(lat, ns):
    """The entry point called through ctypes with plain host arrays."""
    S = (ctypes.c_double * ns)()
    cnt = (ctypes.c_int64 * ns)()
    rc = pss.lib().pss_structure_factor_noalloc(lat._h, 0, S, cnt, ns)
    return rc, np.frombuffer(S, dtype=np.float64).copy(), np.frombuffer(cnt, dtype=np.int64).copy()


@pytest.mark.parametrize("sizes", [((1024, 1024), (256, 256)), ((512, 256), (64, 128)), ((64, 64, 64), (16, 32, 16))])
def test_noalloc_matches_the_allocating_call_twice(sizes):
    for i, n in enumerate(sizes):
        lat = _lattice(n, seed=3 + i, steps=20)
        ns = min(n) // 2 - 1
        S_ref, c_ref = lat.structure_factor(0)
        rc, S, cnt = _raw_noalloc(lat, ns)
        assert rc == 0, pss.lib().pss_last_error()
        assert np.array_equal(cnt, c_ref)
        assert np.all(S_ref > 0)
        assert np.array_equal(S, S_ref)
        # the binding's wrapper gives the same
        S2, c2 = lat.structure_factor_noalloc(0)
        assert np.array_equal(c2, c_ref)
        assert np.array_equal(S2, S_ref)


def test_noalloc_argument_checks():
    lat = _lattice((64, 64), seed=1, steps=2)
    rc, _, _ = _raw_noalloc(lat, 30)  # 31 shells on a 64^2 lattice
    assert rc == -1 and b"n_shells" in pss.lib().pss_last_error()
    S = (ctypes.c_double * 31)()
    cnt = (ctypes.c_int64 * 31)()
    assert pss.lib().pss_structure_factor_noalloc(lat._h, 1, S, cnt, 31) == -1  # no field 1
    assert pss.lib().pss_structure_factor_noalloc(lat._h, 0, None, cnt, 31) == -1
