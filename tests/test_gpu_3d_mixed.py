"""GPU parity of 3D lattices whose sizes are not all powers of two (even
2^a 3^b 5^c on each axis: full complex spectra, one block per line, the
self-sorting radix-4/2/3/5 passes; a z column kernel, y passes and the row
kernel) against the FP64 oracle and numpy's FFT, through the C interface.

Tolerances as on the power-of-two 3D path: transforms within
2e-6 log2(N) of the largest mode; fields within 1e-4 of max(1, max|field|)
after the stated steps (FP32 against FP64); mass within 1e-6 of sum |phi|.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402


def _close(got, want, tol=1e-4, floor=1.0):
    return np.max(np.abs(got - want)) <= tol * max(floor, np.max(np.abs(want)))


@pytest.mark.parametrize("n", [(24, 16, 10), (12, 18, 8), (16, 16, 24), (30, 20, 12)])
def test_transforms_against_numpy(n):
    print(f"mixed 3d transform n={n}", flush=True)
    lat = pss.Lattice(n, dx=(0.7, 1.1, 0.9), dt=0.01, seed=3)
    f, _ = pss.model_b(lat)
    x = np.random.default_rng(sum(n)).normal(size=(n[2], n[1], n[0])).astype(np.float32)
    lat.upload(f, x)
    sp = lat.spectrum(f)
    want = np.fft.fftn(x.astype(np.float64))[:, :, : n[0] // 2 + 1]
    tol = 2e-6 * np.log2(n[0] * n[1] * n[2])
    assert np.max(np.abs(sp - want)) <= tol * np.max(np.abs(want))
    assert np.max(np.abs(lat.download(f) - x)) <= tol * np.max(np.abs(x))


@pytest.mark.parametrize("n,steps", [((24, 24, 24), 40), ((16, 20, 12), 60)])
def test_model_b_matches_oracle(n, steps):
    print(f"mixed 3d model b n={n}", flush=True)
    lat = pss.Lattice(n, dt=0.01, seed=11)
    f, _ = pss.model_b(lat, D=0.01)
    m = om.model_b(OLattice(*n), 0.01, D=0.01, seed=11)
    lat.init_uniform(f, -0.1, 0.1)
    m.init_uniform(0, -0.1, 0.1)
    lat.step(steps)
    m.step(steps)
    assert _close(lat.download(f), m.real(0))
    assert abs(lat.mass(f) - m.state[0][0, 0, 0].real) <= 1e-6 * np.sum(np.abs(m.real(0)))
    S, cnt = lat.structure_factor(f)
    So, no = ob.shell_average(m.lat, ob.structure_factor(m.lat, m.state[0]))
    assert np.array_equal(cnt, no)
    assert np.max(np.abs(S - So)) <= 1e-3 * np.max(So)


def test_two_field_system_matches_oracle():
    n, steps, dt = (24, 20, 16), 40, 0.005
    from paper_2405_02410_amd import Mono
    lat = pss.Lattice(n, dt=dt, seed=2)
    phi = lat.field("phi")
    psi = lat.field("psi")
    lat.term(phi, [Mono(1.0, q2=1), Mono(-1.0, q2=2)], [(phi, 1)], implicit=True)
    lat.term(phi, [Mono(-1.0, q2=1)], [(phi, 3)])
    lat.term(phi, [Mono(-0.15, q2=1)], [(phi, 1), (psi, 2)])
    lat.term(psi, [Mono(0.5), Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    lat.term(psi, [Mono(-1.0)], [(psi, 3)])
    lat.term(psi, [Mono(-0.3)], [(phi, 1), (psi, 1)])
    lat.noise(phi, [Mono(0.005, q2=1)])
    lat.noise(psi, [Mono(0.005)])
    m = om.two_field_3d(OLattice(*n), dt, seed=2)
    for fl in (phi, psi):
        lat.init_uniform(fl, -0.1, 0.1)
    m.init_uniform(0, -0.1, 0.1)
    m.init_uniform(1, -0.1, 0.1)
    lat.step(steps)
    m.step(steps)
    assert _close(lat.download(phi), m.real(0))
    assert _close(lat.download(psi), m.real(1))


def test_model_h_matches_oracle():
    n, steps = (24, 16, 12), 30
    p = dict(a=-1.0, b=1.0, k=1.0, M=1.0, eta=0.5)
    lat = pss.Lattice(n, dt=0.01, seed=7)
    ids, grads = pss.model_h(lat, D=0.01, **p)
    m = om.model_h(OLattice(*n), 0.01, D=0.01, seed=7, **p)
    lat.init_uniform(ids[0], -0.4, 0.4)
    m.init_uniform(0, -0.4, 0.4)
    lat.step(steps)
    m.step(steps)
    for i, fid in enumerate(tuple(ids) + tuple(grads)):
        assert _close(lat.download(fid), m.real(i), floor=1.0 if i == 0 else 0.0), i


def test_lines_per_block_are_bitwise():
    # "tc" (z lines per column block) and "py" (y lines per y-pass block)
    # regroup the same per-line arithmetic
    n = (24, 20, 12)

    def run(**kw):
        lat = pss.Lattice(n, dt=0.01, seed=9)
        f, _ = pss.model_b(lat, D=0.02)
        if kw:
            lat.tune(**kw)
        lat.init_uniform(f, -0.2, 0.2)
        lat.step(20)
        g = lat.geometry()
        return (g["tc"], g["py"]), lat.spectrum(f)

    g0, ref = run()
    assert g0 == (1, 1)
    for kw in (dict(tc=2), dict(py=4), dict(tc=3, py=6), dict(tc=8, py=2)):
        g, sp = run(**kw)
        assert g == (kw.get("tc", 1), kw.get("py", 1))
        assert np.array_equal(sp, ref), kw
