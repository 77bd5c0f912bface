"""GPU parity of 1D lattices whose length is not a power of two (even
N = 2^a 3^b 5^c: self-sorting transforms of radix 4, 2, 3 and 5, the paper's
remark that other sizes are allowed) against the FP64 oracle and numpy's
FFT, through the C interface.

Tolerances as for the power-of-two 1D lattices: transforms within
2e-6 log2(N) of the largest mode; fields within 1e-4 of max(1, max|phi|)
after the stated steps (FP32 against FP64); chunking bitwise.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice, Mono as OMono, fftn  # noqa: E402

SIZES = (12, 96, 120, 160, 250, 1000, 3000)


def _close(got, want, tol=1e-4):
    return np.max(np.abs(got - want)) <= tol * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("n", SIZES)
def test_transforms_against_numpy(n):
    print(f"mixed 1d transform n={n}", flush=True)
    lat = pss.Lattice((n,), dx=(0.7,), dt=0.01, seed=3)
    f, _ = pss.model_b(lat)
    x = np.random.default_rng(n).normal(size=n).astype(np.float32)
    lat.upload(f, x)
    sp = lat.spectrum(f)
    want = np.fft.fft(x.astype(np.float64))[: n // 2 + 1]
    assert np.max(np.abs(sp - want)) <= 2e-6 * np.log2(n) * np.max(np.abs(want))
    back = lat.download(f)
    assert np.max(np.abs(back - x)) <= 2e-6 * np.log2(n) * np.max(np.abs(x))


@pytest.mark.parametrize("n,steps", [(12, 100), (96, 200), (120, 200), (250, 150), (1000, 200), (3000, 100)])
def test_model_b_matches_oracle(n, steps):
    print(f"mixed 1d model b n={n}", flush=True)
    lat = pss.Lattice((n,), dx=(0.9,), dt=0.01, seed=11)
    f, _ = pss.model_b(lat, D=0.01)
    m = om.model_b(OLattice(n, dx=0.9), 0.01, D=0.01, seed=11)
    lat.init_uniform(f, -0.1, 0.1)
    m.init_uniform(0, -0.1, 0.1)
    lat.step(steps)
    m.step(steps)
    assert _close(lat.download(f), m.real(0)[0, 0])
    sp = lat.spectrum(f)
    want = m.state[0][0, 0, : n // 2 + 1]
    assert np.max(np.abs(sp - want)) <= 1e-4 * np.max(np.abs(want))
    assert abs(lat.mass(f) - m.state[0][0, 0, 0].real) <= 1e-6 * np.sum(np.abs(m.real(0)))
    S, cnt = lat.structure_factor(f)
    So, no = ob.shell_average(m.lat, ob.structure_factor(m.lat, m.state[0]))
    assert np.array_equal(cnt, no)
    assert np.max(np.abs(S - So)) <= 1e-3 * np.max(So)


def test_kpz_matches_oracle():
    n = 240
    lat = pss.Lattice((n,), dx=(0.8,), dt=0.01, seed=4)
    f, (g,) = pss.kpz(lat, sigma=1.0, lam=0.5, D=0.01)
    m = om.kpz(OLattice(n, dx=0.8), 0.01, sigma=1.0, lam=0.5, D=0.01, seed=4)
    lat.init_uniform(f, -0.5, 0.5)
    m.init_uniform(0, -0.5, 0.5)
    lat.step(150)
    m.step(150)
    assert _close(lat.download(f), m.real(0)[0, 0])
    assert _close(lat.download(g), m.real(1)[0, 0])


def test_coupled_fields_and_an_intermediate():
    n, dt = 96, 0.005
    lat = pss.Lattice((n,), dt=dt, seed=8)
    m = om.Model(OLattice(n), dt, seed=8)
    ids = []
    for side in ("gpu", "oracle"):
        M_ = Mono if side == "gpu" else OMono
        add = lat.term if side == "gpu" else (lambda t, op, fa, implicit=False: m.add_term(t, op, fa, implicit=implicit))
        fld = lat.field if side == "gpu" else m.add_field
        a = fld("a")
        b = fld("b")
        c = fld("c", dynamic=False)
        add(a, [M_(-0.5), M_(-1.0, q2=1)], [(a, 1)], implicit=True)
        add(b, [M_(-0.2, q2=1), M_(-0.5, q2=2)], [(b, 1)], implicit=True)
        add(c, [M_(1.0, iq=(1, 0, 0))], [(a, 1)])
        add(a, [M_(-1.0)], [(a, 3)])
        add(a, [M_(0.3)], [(b, 1), (c, 1)])
        add(b, [M_(-0.4, q2=1)], [(a, 2)])
        add(b, [M_(0.1)], [(a, 1)])
        ids.append((a, b, c))
    lat.noise(ids[0][0], [Mono(0.004)])
    lat.noise(ids[0][1], [Mono(0.004, q2=1)])
    m.set_noise(ids[1][0], [OMono(0.004)])
    m.set_noise(ids[1][1], [OMono(0.004, q2=1)])
    for fl in ids[0][:2]:
        lat.init_uniform(fl, -0.3, 0.3)
    for fl in ids[1][:2]:
        m.init_uniform(fl, -0.3, 0.3)
    lat.step(120)
    m.step(120)
    for i in range(3):
        assert _close(lat.download(ids[0][i]), m.real(ids[1][i])[0, 0]), i


def test_heat_baths_on_a_mixed_length():
    n, w, dt = 120, 6, 1.0
    lat = pss.Lattice((n,), dt=dt, seed=1)
    f = lat.field("T")
    lat.term(f, [Mono(-1.0, q2=1)], [(f, 1)], implicit=True)
    lat.upload(f, np.full(n, 5.0, dtype=np.float32))
    sites = list(range(w)) + list(range(n - w, n))
    lat.frame(f, sites, [10.0] * w + [0.0] * w)
    m = om.Model(OLattice(n), dt, seed=1)
    g = m.add_field("T")
    m.add_term(g, [OMono(-1.0, q2=1)], [(g, 1)], implicit=True)
    m.set_real(g, np.full(m.lat.shape, 5.0))
    m.set_frame(g, sites, [10.0] * w + [0.0] * w)
    lat.step(200)
    m.step(200)
    assert _close(lat.download(f), m.real(0)[0, 0])


def test_chunking_is_bitwise():
    def mk():
        lat = pss.Lattice((160,), dt=0.01, seed=21)
        f, _ = pss.model_b(lat)
        lat.init_uniform(f, -0.1, 0.1)
        return lat
    a, b = mk(), mk()
    a.step(130)
    for k in (1, 49, 50, 30):
        b.step(k)
    assert np.array_equal(a.spectrum(0), b.spectrum(0))
