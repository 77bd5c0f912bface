"""GPU parity of boundary frames (Sec. "Callback functions": a field held at
fixed values on a band of sites after every step) against the FP64 oracle,
through the C interface; and the paper's heat-bath result on the GPU.

Tolerance: max-abs within 1e-4 of max(1, max|field|) (FP32 against FP64).
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono, PssError  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice, Mono as OMono  # noqa: E402


def _close(got, want, tol=1e-4):
    return np.max(np.abs(got - want)) <= tol * max(1.0, np.max(np.abs(want)))


def _heat(n, dt, w, T1=10.0, T2=0.0):
    lat = pss.Lattice((n,), dt=dt, seed=1)
    f = lat.field("T")
    lat.term(f, [Mono(-1.0, q2=1)], [(f, 1)], implicit=True)
    lat.upload(f, np.full(n, 5.0, dtype=np.float32))
    sites = list(range(w)) + list(range(n - w, n))
    lat.frame(f, sites, [T1] * w + [T2] * w)
    m = om.Model(OLattice(n), dt, seed=1)
    g = m.add_field("T")
    m.add_term(g, [OMono(-1.0, q2=1)], [(g, 1)], implicit=True)
    m.set_real(g, np.full(m.lat.shape, 5.0))
    m.set_frame(g, sites, [T1] * w + [T2] * w)
    return lat, m


def test_heat_baths_1d_match_the_oracle_and_reach_the_line():
    n, w = 256, 10
    lat, m = _heat(n, 1.0, w)
    lat.step(300)
    m.step(300)
    assert _close(lat.download(0), m.real(0)[0, 0])
    lat.step(19700)
    x = np.arange(n)
    line = 10.0 + (0.0 - 10.0) * (x - (w - 1)) / ((n - w) - (w - 1))
    got = lat.download(0)
    # the baths hold (up to the FP32 round trip of the download)
    assert np.max(np.abs(got[:w] - 10.0)) <= 1e-5 * 10.0 and np.max(np.abs(got[n - w:])) <= 1e-5 * 10.0
    assert np.max(np.abs(got[w:n - w] - line[w:n - w])) <= 0.02 * 10.0


def _model_b_framed(n, seed, sites, values):
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    f, _ = pss.model_b(lat)
    lat.init_uniform(f, -0.1, 0.1)
    lat.frame(f, sites, values)
    olat = OLattice(*n) if len(n) == 3 else OLattice(n[0], n[1], 1)
    m = om.model_b(olat, 0.01, seed=seed)
    m.init_uniform(0, -0.1, 0.1)
    m.set_frame(0, sites, values)
    return lat, m


@pytest.mark.parametrize("n", [(64, 32), (16, 16, 16)])
def test_model_b_with_a_frame_matches_the_oracle(n):
    print(f"frame n={n}", flush=True)
    nx = n[0]
    sites = np.array([i for i in range(int(np.prod(n))) if (i % nx) < 3])  # a band x < 3
    values = np.full(sites.size, 0.4, dtype=np.float32)
    lat, m = _model_b_framed(n, 7, sites, values)
    lat.step(60)
    m.step(60)
    want = m.real(0)
    want = want[0] if len(n) == 2 else want
    got = lat.download(0)
    assert _close(got, want)
    assert np.max(np.abs(got.reshape(-1)[sites] - 0.4)) <= 1e-5  # the frame holds (FP32 round trip)


def test_frame_removed_and_changed_between_steps():
    n = (32, 32)
    sites = np.arange(32)  # the row y = 0
    lat, m = _model_b_framed(n, 3, sites, np.full(32, -0.2, dtype=np.float32))
    lat.step(10)
    m.step(10)
    lat.frame(0, [], [])  # removed: plain steps again (graphs rebuilt)
    m.frames.clear()
    lat.step(10)
    m.step(10)
    s2 = np.arange(32) * 32  # the column x = 0
    lat.frame(0, s2, np.full(32, 0.3, dtype=np.float32))
    m.set_frame(0, s2, np.full(32, 0.3))
    lat.step(15)
    m.step(15)
    assert _close(lat.download(0), m.real(0)[0])


def test_framed_lattices_stay_out_of_batches_and_the_adjoint():
    lat = pss.Lattice((64, 64), dt=0.01, seed=1)
    f, _ = pss.model_b(lat)
    lat.init_uniform(f)
    other = pss.Lattice((64, 64), dt=0.01, seed=2)
    pss.model_b(other)
    lat.frame(f, [0, 1], [0.0, 0.0])
    with pytest.raises(PssError) as e:
        pss.Batch([lat, other])
    assert e.value.name == "PSS_E_UNSUPPORTED"
    with pytest.raises(PssError):
        lat.adjoint_model_b(10, np.zeros(31), ckpt_every=5)
    lat.frame(f, [], [])
    b = pss.Batch([lat, other])
    with pytest.raises(PssError) as e:
        lat.frame(f, [0], [1.0])
    assert e.value.name == "PSS_E_STATE"
    b.close()


@pytest.mark.parametrize("n", [(64, 32), (16, 16, 16)])
def test_framed_steps_chunk_bitwise(n):
    # a framed step runs the update launch, the frame and the rebuilt
    # products; the step counter then moves on once per chunk
    nx = n[0]
    sites = np.array([i for i in range(int(np.prod(n))) if (i % nx) < 2])
    values = np.full(sites.size, -0.3, dtype=np.float32)

    def mk():
        lat = pss.Lattice(n, dt=0.01, seed=13)
        f, _ = pss.model_b(lat, D=0.02)
        lat.init_uniform(f, -0.1, 0.1)
        lat.frame(f, sites, values)
        return lat

    a, b = mk(), mk()
    a.step(75)
    for k in (10, 50, 15):
        b.step(k)
    assert a.step_index == b.step_index == 75
    assert np.array_equal(a.spectrum(0), b.spectrum(0))
