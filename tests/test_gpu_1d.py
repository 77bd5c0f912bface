"""GPU parity of 1D lattices (one block holds the whole line; full complex
spectrum in natural mode order) against the FP64 oracle, through the C
interface.

Tolerances as in 2D: real-space fields within 1e-4 of max(1, max|phi|) after
the stated steps (FP32 against FP64), 1e-5 relative for single transforms and
a few steps; chunking, restarts and state loads bitwise.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono, PssError  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice, Mono as OMono, fftn  # noqa: E402

TOL = 1e-4


def _close(got, want, tol=TOL):
    return np.max(np.abs(got - want)) <= tol * max(1.0, np.max(np.abs(want)))


def _model_b_pair(n, dx, seed, D=0.01, dt=0.01):
    lat = pss.Lattice((n,), dx=(dx,), dt=dt, seed=seed)
    f, _ = pss.model_b(lat, D=D)
    m = om.model_b(OLattice(n, dx=dx), dt, D=D, seed=seed)
    lat.init_uniform(f, -0.1, 0.1)
    m.init_uniform(0, -0.1, 0.1)
    return lat, m


@pytest.mark.parametrize("n,steps", [(8, 100), (64, 200), (256, 200), (1024, 200), (4096, 100)])
def test_model_b_1d_matches_oracle(n, steps):
    print(f"1d model b n={n}", flush=True)
    lat, m = _model_b_pair(n, 0.9, seed=11)
    # the same initial field on both sides (the download is one FP32 round trip)
    assert _close(lat.download(0), m.real(0)[0, 0], 1e-6)
    lat.step(steps)
    m.step(steps)
    assert lat.step_index == steps
    assert _close(lat.download(0), m.real(0)[0, 0])
    # the spectrum (modes 0 .. N/2) and the mass
    sp = lat.spectrum(0)
    want = m.state[0][0, 0, : n // 2 + 1]
    assert np.max(np.abs(sp - want)) <= 1e-4 * np.max(np.abs(want))
    assert abs(lat.mass(0) - m.state[0][0, 0, 0].real) <= 1e-6 * np.sum(np.abs(m.real(0)))


def test_kpz_1d_matches_oracle():
    n, dx, dt = 512, 0.8, 0.01
    lat = pss.Lattice((n,), dx=(dx,), dt=dt, seed=4)
    f, (g,) = pss.kpz(lat, sigma=1.0, lam=0.5, D=0.01)
    m = om.kpz(OLattice(n, dx=dx), dt, sigma=1.0, lam=0.5, D=0.01, seed=4)
    lat.init_uniform(f, -0.5, 0.5)
    m.init_uniform(0, -0.5, 0.5)
    lat.step(150)
    m.step(150)
    assert _close(lat.download(f), m.real(0)[0, 0])
    assert _close(lat.download(g), m.real(1)[0, 0])  # the gradient, computed on the device


def test_coupled_fields_1d():
    # two fields, products of both, a linear coupling and an intermediate
    # with an odd operator: the 1D kernel's general path with two fields
    n, dt = 128, 0.005
    lat = pss.Lattice((n,), dt=dt, seed=8)
    m = om.Model(OLattice(n), dt, seed=8)
    ids = []
    for side in ("gpu", "oracle"):
        M_ = Mono if side == "gpu" else OMono
        add = lat.term if side == "gpu" else (lambda t, op, fa, implicit=False: m.add_term(t, op, fa, implicit=implicit))
        fld = lat.field if side == "gpu" else m.add_field
        a = fld("a")
        b = fld("b")
        c = fld("c", dynamic=False) if side == "gpu" else m.add_field("c", dynamic=False)
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


def test_upload_download_and_structure_factor_1d():
    n = 256
    lat = pss.Lattice((n,), dx=(0.5,), dt=0.01, seed=2)
    f, _ = pss.model_b(lat)
    x = np.random.default_rng(5).normal(size=n).astype(np.float32)
    lat.upload(f, x)
    assert np.max(np.abs(lat.download(f) - x)) <= 1e-6 * np.max(np.abs(x))
    sp = lat.spectrum(f)
    want = np.fft.fft(x.astype(np.float64))[: n // 2 + 1]
    assert np.max(np.abs(sp - want)) <= 2e-6 * 8 * np.max(np.abs(want))
    S, cnt = lat.structure_factor(f)
    olat = OLattice(n, dx=0.5)
    So, no = ob.shell_average(olat, ob.structure_factor(olat, fftn(x.astype(np.complex128).reshape(olat.shape))))
    assert np.array_equal(cnt, no)
    assert np.max(np.abs(S - So)) <= 1e-5 * np.max(So)


def test_chunking_restart_and_state_load_are_bitwise_1d():
    def mk():
        lat = pss.Lattice((512,), dt=0.01, seed=21)
        f, _ = pss.model_b(lat)
        lat.init_uniform(f, -0.1, 0.1)
        return lat
    a, b, c = mk(), mk(), mk()
    a.step(130)
    for k in (1, 49, 50, 30):
        b.step(k)
    assert np.array_equal(a.spectrum(0), b.spectrum(0))
    c.step(60)
    blob = c.save()
    c.step(70)
    assert np.array_equal(a.spectrum(0), c.spectrum(0))
    c.load(blob)
    c.step(70)
    assert np.array_equal(a.spectrum(0), c.spectrum(0))
    assert c.kernels_per_step() == 1


def test_nonfinite_flag_and_refusals_1d():
    lat = pss.Lattice((64,), dt=0.01, seed=1)
    f, _ = pss.model_b(lat)
    bad = np.zeros(64, dtype=np.float32)
    bad[5] = np.nan
    lat.upload(f, bad)
    lat.step(2)
    with pytest.raises(PssError) as e:
        lat.sync()
    assert e.value.name == "PSS_E_NONFINITE"
    lat.sync()  # reported once
    other = pss.Lattice((64,), dt=0.01, seed=2)
    pss.model_b(other)
    with pytest.raises(PssError) as e:
        pss.Batch([lat, other])
    assert e.value.name == "PSS_E_UNSUPPORTED"
