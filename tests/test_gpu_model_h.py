"""GPU parity of Model H (pss.model_h; 2D: order parameter, two velocity
components, two gradient intermediates, five product channels over five
factor slots; 3D: three of each, eight channels over seven slots) against the
FP64 oracle, through the C interface.

Tolerance: every field within 1e-4 of its largest magnitude (and of 1 for
the order parameter) after the stated steps, FP32 against FP64, the bar of
the other multi-field models; the mean of phi within 1e-6 of sum |phi|; the
discrete divergence of the flow off the Nyquist planes within 1e-5 of
|q||v| (FP32 rounding of a quantity that is zero in exact arithmetic).
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402

PARAMS = dict(a=-1.0, b=1.0, k=1.0, M=1.0, eta=0.5)


def _pair(n, dx, seed, D=0.01, dt=0.01, **kw):
    p = dict(PARAMS, **kw)
    lat = pss.Lattice(n, dx=dx, dt=dt, seed=seed)
    (f, vx, vy), (gx, gy) = pss.model_h(lat, D=D, **p)
    m = om.model_h(OLattice(n[0], n[1], 1, dx=dx[0], dy=dx[1]), dt, D=D, seed=seed, **p)
    lat.init_uniform(f, -0.4, 0.4)
    m.init_uniform(0, -0.4, 0.4)
    return lat, m, (f, vx, vy, gx, gy)


def _close(got, want, floor=0.0, tol=1e-4):
    scale = max(floor, float(np.max(np.abs(want))))
    return float(np.max(np.abs(got - want))) <= tol * scale, float(np.max(np.abs(got - want))) / scale


@pytest.mark.parametrize("n,dx,steps", [((64, 64), (1.0, 1.0), 150), ((128, 64), (0.8, 1.1), 100),
                                        ((256, 256), (1.0, 1.0), 100), ((32, 128), (1.0, 0.7), 120)])
def test_model_h_matches_oracle(n, dx, steps):
    print(f"model h n={n} dx={dx} steps={steps}", flush=True)
    lat, m, ids = _pair(n, dx, seed=6)
    lat.step(steps)
    m.step(steps)
    assert lat.step_index == steps
    for i, fid in enumerate(ids):
        want = m.real(i)[0]
        got = lat.download(fid)
        ok, err = _close(got, want, floor=1.0 if i == 0 else 0.0)
        assert ok, (i, err)
    # the flow is not trivially small: the interfaces drive it
    assert np.max(np.abs(m.real(1))) > 1e-3


def test_model_h_full_size_and_invariants():
    n, steps = (512, 512), 20
    print(f"model h n={n} steps={steps}", flush=True)
    lat, m, ids = _pair(n, (1.0, 1.0), seed=2, D=0.02)
    mass0 = lat.mass(ids[0])
    lat.step(steps)
    m.step(steps)
    for i, fid in enumerate(ids[:3]):
        ok, err = _close(lat.download(fid), m.real(i)[0], floor=1.0 if i == 0 else 0.0)
        assert ok, (i, err)
    phi = lat.download(ids[0])
    assert abs(lat.mass(ids[0]) - mass0) <= 1e-6 * np.sum(np.abs(phi))
    # divergence of the device flow, off the Nyquist planes
    sx = lat.spectrum(ids[1]).astype(np.complex128)[: n[1], :]
    sy = lat.spectrum(ids[2]).astype(np.complex128)[: n[1], :]
    kx = np.arange(n[0] // 2 + 1)
    ky = np.where(np.arange(n[1]) < n[1] // 2, np.arange(n[1]), np.arange(n[1]) - n[1])
    qx = 2 * np.pi * kx[None, :] / n[0]
    qy = 2 * np.pi * ky[:, None] / n[1]
    keep = (kx[None, :] != n[0] // 2) & (ky[:, None] != -(n[1] // 2))
    div = 1j * qx * sx + 1j * qy * sy
    scale = np.max(np.sqrt(qx ** 2 + qy ** 2) * (np.abs(sx) + np.abs(sy)))
    assert scale > 0
    assert np.max(np.abs(div[keep])) <= 1e-5 * scale


def test_flat_profile_drives_no_flow():
    n, dt = (128, 32), 0.01
    lat = pss.Lattice(n, dt=dt, seed=3)
    (f, vx, vy), _ = pss.model_h(lat, D=0.0, **PARAMS)
    prof = np.random.default_rng(1).uniform(-0.5, 0.5, size=n[0]).astype(np.float32)
    lat.upload(f, np.broadcast_to(prof[None, :], (n[1], n[0])).copy())
    ref = pss.Lattice(n, dt=dt, seed=3)
    g, _ = pss.model_b(ref, a=PARAMS["M"] * PARAMS["a"], b=PARAMS["M"] * PARAMS["b"], k=PARAMS["M"] * PARAMS["k"],
                       D=0.0)
    ref.upload(g, np.broadcast_to(prof[None, :], (n[1], n[0])).copy())
    lat.step(80)
    ref.step(80)
    assert np.max(np.abs(lat.download(vx))) <= 1e-6
    assert np.max(np.abs(lat.download(vy))) <= 1e-6
    ok, err = _close(lat.download(f), ref.download(g), floor=1.0, tol=1e-5)
    assert ok, err


def test_model_h_restart_and_chunking_bitwise():
    def mk():
        lat = pss.Lattice((128, 128), dt=0.01, seed=12)
        (f, vx, vy), _ = pss.model_h(lat, D=0.01, **PARAMS)
        lat.init_uniform(f, -0.4, 0.4)
        return lat, (f, vx, vy)
    (a, ids), (b, _) = mk(), mk()
    a.step(75)
    for k in (10, 50, 15):
        b.step(k)
    for fid in ids:
        assert np.array_equal(a.spectrum(fid), b.spectrum(fid))


@pytest.mark.parametrize("n,steps", [((16, 16, 16), 60), ((32, 16, 8), 40), ((32, 32, 32), 30)])
def test_model_h_3d_matches_oracle(n, steps):
    # four dynamic fields, three gradient intermediates, seven factor slots;
    # the six stress products each feed all three velocity components
    print(f"model h 3d n={n} steps={steps}", flush=True)
    lat = pss.Lattice(n, dt=0.01, seed=7)
    ids, grads = pss.model_h(lat, D=0.01, **PARAMS)
    m = om.model_h(OLattice(*n), 0.01, D=0.01, seed=7, **PARAMS)
    lat.init_uniform(ids[0], -0.4, 0.4)
    m.init_uniform(0, -0.4, 0.4)
    lat.step(steps)
    m.step(steps)
    for i, fid in enumerate(tuple(ids) + tuple(grads)):
        ok, err = _close(lat.download(fid), m.real(i), floor=1.0 if i == 0 else 0.0)
        assert ok, (i, err)
    assert np.max(np.abs(m.real(1))) > 1e-4


def test_model_h_3d_invariants():
    n, steps = (64, 64, 64), 20
    print(f"model h 3d n={n} steps={steps}", flush=True)
    lat = pss.Lattice(n, dt=0.01, seed=5)
    ids, _ = pss.model_h(lat, D=0.02, **PARAMS)
    lat.init_uniform(ids[0], -0.4, 0.4)
    mass0 = lat.mass(ids[0])
    lat.step(steps)
    phi = lat.download(ids[0])
    assert np.all(np.isfinite(phi))
    assert abs(lat.mass(ids[0]) - mass0) <= 1e-6 * np.sum(np.abs(phi))
    sp = [lat.spectrum(v).astype(np.complex128) for v in ids[1:]]  # (z, y, kx)
    kx = np.arange(n[0] // 2 + 1)[None, None, :]
    ky = np.where(np.arange(n[1]) < n[1] // 2, np.arange(n[1]), np.arange(n[1]) - n[1])[None, :, None]
    kz = np.where(np.arange(n[2]) < n[2] // 2, np.arange(n[2]), np.arange(n[2]) - n[2])[:, None, None]
    q = [2 * np.pi * kx / n[0], 2 * np.pi * ky / n[1], 2 * np.pi * kz / n[2]]
    keep = (kx != n[0] // 2) & (ky != -(n[1] // 2)) & (kz != -(n[2] // 2))
    div = sum(1j * q[c] * sp[c] for c in range(3))
    scale = np.max(np.sqrt(q[0] ** 2 + q[1] ** 2 + q[2] ** 2) * sum(np.abs(s) for s in sp))
    assert scale > 0
    assert np.max(np.abs(div[np.broadcast_to(keep, div.shape)])) <= 1e-5 * scale
