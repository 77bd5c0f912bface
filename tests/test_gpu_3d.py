"""GPU parity of the 3D path (z update kernel, y passes, x kernel) against the
FP64 oracle, through the C interface."""

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice, Mono as OMono  # noqa: E402


def _half(full):
    return full[..., : full.shape[-1] // 2 + 1]


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(1e-30, np.max(np.abs(b)))


@pytest.mark.parametrize("n", [(8, 8, 8), (16, 8, 32), (32, 16, 8), (64, 64, 64), (8, 128, 16), (256, 256, 256)])
def test_3d_transform_round_trip(n):
    lat = pss.Lattice(n, dt=0.01)
    lat.field("phi")
    shape = tuple(reversed(n))
    x = inputs.random_field(shape, seed=sum(n), amp=1.0)
    lat.upload(0, x)
    ref = _half(np.fft.fftn(x.astype(np.float64)))
    assert _rel(lat.spectrum(0), ref) < 3e-6 * np.log2(max(n))
    back = lat.download(0)
    assert np.max(np.abs(back - x)) < 3e-6 * np.log2(max(n)) * np.max(np.abs(x))


def _pair(n, dt=0.005, seed=1, D=0.005, c=-0.5, g=0.3):
    a, b, k = -1.0, 1.0, 1.0
    lat = pss.Lattice(n, dt=dt, seed=seed)
    phi = lat.field("phi")
    psi = lat.field("psi")
    lat.term(phi, [Mono(-a, q2=1), Mono(-k, q2=2)], [(phi, 1)], implicit=True)
    lat.term(phi, [Mono(-b, q2=1)], [(phi, 3)])
    lat.term(phi, [Mono(-0.5 * g, q2=1)], [(phi, 1), (psi, 2)])
    lat.term(psi, [Mono(-c), Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    lat.term(psi, [Mono(-1.0)], [(psi, 3)])
    lat.term(psi, [Mono(-g)], [(phi, 1), (psi, 1)])
    if D:
        lat.noise(phi, [Mono(D, q2=1)])
        lat.noise(psi, [Mono(D)])
    lat.init_uniform(phi)
    lat.init_uniform(psi)
    m = om.two_field_3d(OLattice(*n), dt, a=a, b=b, k=k, c=c, g=g, D=D, seed=seed)
    m.init_uniform(0, -0.1, 0.1)
    m.init_uniform(1, -0.1, 0.1)
    return lat, m


@pytest.mark.parametrize("n", [(16, 16, 16), (32, 32, 32), (16, 8, 32), (32, 16, 8)])
def test_3d_two_field_matches_oracle(n):
    lat, m = _pair(n)
    lat.step(30)
    m.step(30)
    for f in (0, 1):
        assert np.max(np.abs(lat.download(f) - m.real(f))) < 2e-5
        assert _rel(lat.spectrum(f), _half(m.state[f])) < 1e-4


def test_3d_32_cubed_100_steps_and_mass():
    lat, m = _pair((32, 32, 32))
    mass0 = lat.mass(0)
    lat.step(100)
    m.step(100)
    for f in (0, 1):
        assert np.max(np.abs(lat.download(f) - m.real(f))) < 1e-4
    phi = lat.download(0)
    assert abs(lat.mass(0) - mass0) <= 1e-6 * np.sum(np.abs(phi))


def test_3d_model_b_single_field_and_noise():
    n = (16, 32, 16)
    lat = pss.Lattice(n, dt=0.01, seed=7)
    f, _ = pss.model_b(lat, D=0.05)
    lat.init_uniform(f)
    m = om.model_b(OLattice(*n), 0.01, D=0.05, seed=7)
    m.init_uniform(0, -0.1, 0.1)
    lat.step(40)
    m.step(40)
    assert np.max(np.abs(lat.download(f) - m.real(0))) < 2e-5
    S, cnt = lat.structure_factor(f)
    so, no = ob.shell_average(m.lat, ob.structure_factor(m.lat, m.state[0]))
    assert np.array_equal(cnt, no)
    assert _rel(S, so) < 1e-4


def test_3d_direct_terms():
    n, dt = (16, 16, 8), 0.02
    lat = pss.Lattice(n, dt=dt)
    a = lat.field("a")
    b = lat.field("b")
    lat.term(a, [Mono(-1.0, q2=1)], [(a, 1)], implicit=True)
    lat.term(b, [Mono(-0.5), Mono(-2.0, q2=1)], [(b, 1)], implicit=True)
    lat.term(a, [Mono(0.7, iq=(0, 0, 1))], [(b, 1)])
    lat.term(b, [Mono(-0.4, q2=1)], [(a, 1)])
    xa = inputs.random_field((8, 16, 16), seed=4)
    xb = inputs.random_field((8, 16, 16), seed=5)
    lat.upload(a, xa)
    lat.upload(b, xb)
    lat.step(20)
    m = om.Model(OLattice(*n), dt)
    A = m.add_field("a")
    B = m.add_field("b")
    m.add_term(A, [OMono(-1.0, q2=1)], [(A, 1)], implicit=True)
    m.add_term(B, [OMono(-0.5), OMono(-2.0, q2=1)], [(B, 1)], implicit=True)
    m.add_term(A, [OMono(0.7, iq=(0, 0, 1))], [(B, 1)])
    m.add_term(B, [OMono(-0.4, q2=1)], [(A, 1)])
    m.set_real(A, xa)
    m.set_real(B, xb)
    m.step(20)
    assert _rel(lat.spectrum(a), _half(m.state[A])) < 1e-5
    assert _rel(lat.spectrum(b), _half(m.state[B])) < 1e-5


def test_3d_restart_is_bitwise():
    a, _ = _pair((16, 16, 16), seed=3, D=0.02)
    a.step(40)
    ref = a.spectrum(1)
    b, _ = _pair((16, 16, 16), seed=3, D=0.02)
    b.step(15)
    blob = b.save()
    c, _ = _pair((16, 16, 16), seed=3, D=0.02)
    c.load(blob)
    c.step(25)
    assert np.array_equal(c.spectrum(1), ref)
