"""GPU parity of 2D lattices whose sizes are not both powers of two (even
2^a 3^b 5^c on each axis: full complex spectra, one block per line, the
self-sorting radix-4/2/3/5 passes) against the FP64 oracle and numpy's FFT,
through the C interface.

Tolerances as on the power-of-two path: transforms within 2e-6 log2(N) of
the largest mode; fields within 1e-4 of max(1, max|field|) after the stated
steps (FP32 against FP64); mass within 1e-6 of sum |phi|; chunking bitwise.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import PssError  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402


def _close(got, want, tol=1e-4, floor=1.0):
    return np.max(np.abs(got - want)) <= tol * max(floor, np.max(np.abs(want)))


@pytest.mark.parametrize("n", [(96, 64), (64, 96), (120, 90), (250, 24)])
def test_transforms_against_numpy(n):
    print(f"mixed 2d transform n={n}", flush=True)
    lat = pss.Lattice(n, dx=(0.7, 1.1), dt=0.01, seed=3)
    f, _ = pss.model_b(lat)
    x = np.random.default_rng(n[0] + n[1]).normal(size=(n[1], n[0])).astype(np.float32)
    lat.upload(f, x)
    sp = lat.spectrum(f)
    want = np.fft.fft2(x.astype(np.float64))[:, : n[0] // 2 + 1]
    tol = 2e-6 * np.log2(n[0] * n[1])
    assert np.max(np.abs(sp - want)) <= tol * np.max(np.abs(want))
    assert np.max(np.abs(lat.download(f) - x)) <= tol * np.max(np.abs(x))


@pytest.mark.parametrize("n,steps", [((96, 96), 100), ((120, 64), 100), ((90, 160), 80)])
def test_model_b_matches_oracle(n, steps):
    print(f"mixed 2d model b n={n}", flush=True)
    lat = pss.Lattice(n, dx=(0.9, 0.9), dt=0.01, seed=11)
    f, _ = pss.model_b(lat, D=0.01)
    m = om.model_b(OLattice(n[0], n[1], 1, dx=0.9, dy=0.9), 0.01, D=0.01, seed=11)
    lat.init_uniform(f, -0.1, 0.1)
    m.init_uniform(0, -0.1, 0.1)
    lat.step(steps)
    m.step(steps)
    assert _close(lat.download(f), m.real(0)[0])
    sp = lat.spectrum(f)
    want = m.state[0][0][:, : n[0] // 2 + 1]
    assert np.max(np.abs(sp - want)) <= 1e-4 * np.max(np.abs(want))
    assert abs(lat.mass(f) - m.state[0][0, 0, 0].real) <= 1e-6 * np.sum(np.abs(m.real(0)))
    S, cnt = lat.structure_factor(f)
    So, no = ob.shell_average(m.lat, ob.structure_factor(m.lat, m.state[0]))
    assert np.array_equal(cnt, no)
    assert np.max(np.abs(S - So)) <= 1e-3 * np.max(So)


def test_model_h_matches_oracle():
    # three fields, gradient intermediates, shared channels, general operators
    n, steps = (96, 96), 60
    p = dict(a=-1.0, b=1.0, k=1.0, M=1.0, eta=0.5)
    lat = pss.Lattice(n, dt=0.01, seed=6)
    ids, grads = pss.model_h(lat, D=0.01, **p)
    m = om.model_h(OLattice(n[0], n[1], 1), 0.01, D=0.01, seed=6, **p)
    lat.init_uniform(ids[0], -0.4, 0.4)
    m.init_uniform(0, -0.4, 0.4)
    lat.step(steps)
    m.step(steps)
    for i, fid in enumerate(tuple(ids) + tuple(grads)):
        assert _close(lat.download(fid), m.real(i)[0], floor=1.0 if i == 0 else 0.0), i


def test_frame_on_a_mixed_lattice():
    n = (96, 64)
    lat = pss.Lattice(n, dt=0.01, seed=5)
    f, _ = pss.model_b(lat)
    lat.init_uniform(f, -0.1, 0.1)
    sites = [y * n[0] + x for y in range(n[1]) for x in range(4)]
    values = [0.2] * len(sites)
    lat.frame(f, sites, values)
    m = om.model_b(OLattice(n[0], n[1], 1), 0.01, seed=5)
    m.init_uniform(0, -0.1, 0.1)
    m.set_frame(0, sites, values)
    lat.step(60)
    m.step(60)
    assert _close(lat.download(f), m.real(0)[0])


def test_chunking_is_bitwise_and_refusals():
    def mk():
        lat = pss.Lattice((120, 96), dt=0.01, seed=21)
        f, _ = pss.model_b(lat)
        lat.init_uniform(f, -0.1, 0.1)
        return lat
    a, b = mk(), mk()
    a.step(130)
    for k in (1, 49, 50, 30):
        b.step(k)
    assert np.array_equal(a.spectrum(0), b.spectrum(0))
    with pytest.raises(PssError) as e:
        a.time_kernel(0, 5)
    assert e.value.name == "PSS_E_UNSUPPORTED"
    with pytest.raises(PssError) as e:
        pss.Batch([a, b])
    assert e.value.name == "PSS_E_UNSUPPORTED"


def test_lines_per_block_are_bitwise_and_checked():
    # pss_tuning_set "tc": neighbouring column lines per block only regroup
    # the same per-line arithmetic
    n = (120, 96)

    def run(tc):
        lat = pss.Lattice(n, dt=0.01, seed=8)
        f, _ = pss.model_b(lat, D=0.02)
        if tc:
            lat.tune(tc=tc)
        lat.init_uniform(f, -0.2, 0.2)
        lat.step(40)
        return lat.geometry()["tc"], lat.spectrum(f)

    tc0, ref = run(None)
    assert tc0 == 1
    for tc in (2, 3, 8):
        got_tc, sp = run(tc)
        assert got_tc == tc
        assert np.array_equal(sp, ref), tc
    lat = pss.Lattice(n, dt=0.01, seed=8)
    pss.model_b(lat)
    lat.tune(tc=7)  # not a divisor of Nx
    with pytest.raises(PssError) as e:
        lat.init_uniform(0, -0.1, 0.1)
    assert e.value.name == "PSS_E_UNSUPPORTED"
