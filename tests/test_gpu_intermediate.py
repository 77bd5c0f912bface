"""GPU parity of intermediate (non-dynamic) fields (Sec. "Writing models")
and of the KPZ equation built from them (Sec. "What cuPSS calculates"),
through the C interface, against the FP64 oracle.

An intermediate field psi = sum_k op_k phi_k / (1 - L_psi) is evaluated in the
update kernel from the fields' values at each mode: from the new state for the
factors of the next products, and from the step-n state inside linear terms.
Tolerance: max-abs of the real-space fields within 1e-4 of max(1, max|field|)
after 100 steps in 2D (FP32 against FP64, as for Model B), 50 steps in 3D;
downloaded intermediates within the same bound.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice, Mono as OMono  # noqa: E402

TOL = 1e-4


def _olat(n, dx):
    if len(n) == 2:
        return OLattice(n[0], n[1], 1, dx=dx[0], dy=dx[1])
    return OLattice(n[0], n[1], n[2], dx=dx[0], dy=dx[1], dz=dx[2])


def _real(m, f, n):
    r = m.real(f)
    return r[0] if len(n) == 2 else r


def _close(got, want):
    return np.max(np.abs(got - want)) <= TOL * max(1.0, np.max(np.abs(want)))


def _kpz_pair(n, dx, seed, sigma=1.0, lam=0.5, D=0.01, dt=0.01):
    lat = pss.Lattice(n, dx=dx, dt=dt, seed=seed)
    f, grads = pss.kpz(lat, sigma=sigma, lam=lam, D=D)
    m = om.kpz(_olat(n, dx), dt, sigma=sigma, lam=lam, D=D, seed=seed)
    lat.init_uniform(f, -0.5, 0.5)
    m.init_uniform(0, -0.5, 0.5)
    return lat, m, f, grads


@pytest.mark.parametrize("n,dx,steps", [((64, 64), (0.8, 0.8), 100), ((128, 32), (1.0, 0.6), 100),
                                        ((16, 16, 32), (1.0, 1.0, 0.8), 50), ((32, 16, 16), (0.9, 1.0, 1.0), 50)])
def test_kpz_matches_oracle(n, dx, steps):
    print(f"kpz n={n} steps={steps}", flush=True)
    lat, m, f, grads = _kpz_pair(n, dx, seed=21)
    lat.step(steps)
    m.step(steps)
    assert lat.step_index == steps
    assert _close(lat.download(f), _real(m, 0, n))
    # the gradient intermediates, computed on the device from the state
    for i, g in enumerate(grads):
        assert _close(lat.download(g), _real(m, 1 + i, n)), i


def test_kpz_noise_free_single_step_is_the_closed_form():
    # one step from A cos(qx x) + B cos(qy y) (the oracle's pinned closed form,
    # re-evaluated here in real space): modes 0, qx, qy, 2 qx, 2 qy
    n, dx, dt, sigma, lam = (32, 32), (0.9, 0.9), 0.02, 1.3, 0.7
    lat = pss.Lattice(n, dx=dx, dt=dt, seed=1)
    f, _ = pss.kpz(lat, sigma=sigma, lam=lam, D=0.0)
    kx, ky, A, B = 2, 3, 0.4, 0.25
    x = np.arange(32) * 0.9
    qx, qy = 2 * np.pi * kx / (32 * 0.9), 2 * np.pi * ky / (32 * 0.9)
    phi0 = A * np.cos(qx * x)[None, :] + B * np.cos(qy * x)[:, None]
    lat.upload(f, phi0.astype(np.float32))
    lat.step(1)
    ax, ay = lam * A * A * qx * qx / 2, lam * B * B * qy * qy / 2
    want = (A * np.cos(qx * x)[None, :] / (1 + dt * sigma * qx * qx)
            + B * np.cos(qy * x)[:, None] / (1 + dt * sigma * qy * qy) + dt * (ax + ay)
            - dt * ax * np.cos(2 * qx * x)[None, :] / (1 + dt * sigma * 4 * qx * qx)
            - dt * ay * np.cos(2 * qy * x)[:, None] / (1 + dt * sigma * 4 * qy * qy))
    assert np.max(np.abs(lat.download(f) - want)) <= 2e-6


def _paper_pair(n, dx, seed, dt=0.005):
    """Model B with the paper's intermediate psi + psi q^2 = -q^2 phi entering
    a product (g psi phi) and a linear term (-0.8 psi)."""
    a, b, k, g, D = -1.0, 1.0, 1.0, 0.4, 0.005
    lat = pss.Lattice(n, dx=dx, dt=dt, seed=seed)
    m = om.Model(_olat(n, dx), dt, seed=seed)
    f = lat.field("phi")
    p = lat.field("psi", dynamic=False)
    fo = m.add_field("phi")
    po = m.add_field("psi", dynamic=False)
    for L_, M_ in ((lat, Mono), (m, OMono)):
        fld, psi = (f, p) if L_ is lat else (fo, po)
        add = L_.term if L_ is lat else (lambda t, op, fa, implicit=False: m.add_term(t, op, fa, implicit=implicit))
        add(fld, [M_(-a, q2=1), M_(-k, q2=2)], [(fld, 1)], implicit=True)
        add(fld, [M_(-b, q2=1)], [(fld, 3)])
        add(psi, [M_(-1.0, q2=1)], [(psi, 1)], implicit=True)
        add(psi, [M_(-1.0, q2=1)], [(fld, 1)])
        add(fld, [M_(g)], [(psi, 1), (fld, 1)])
        add(fld, [M_(-0.8)], [(psi, 1)])
    lat.noise(f, [Mono(D, q2=1)])
    m.set_noise(fo, [OMono(D, q2=1)])
    lat.init_uniform(f, -0.2, 0.2)
    m.init_uniform(fo, -0.2, 0.2)
    return lat, m, f, p


@pytest.mark.parametrize("n,dx,steps", [((64, 32), (1.0, 0.7), 100), ((16, 32, 16), (1.0, 1.0, 1.0), 50)])
def test_paper_intermediate_in_products_and_linear_terms(n, dx, steps):
    print(f"paper intermediate n={n}", flush=True)
    lat, m, f, p = _paper_pair(n, dx, seed=5)
    assert _close(lat.download(p), _real(m, 1, n))  # before any step
    lat.step(steps)
    m.step(steps)
    assert _close(lat.download(f), _real(m, 0, n))
    assert _close(lat.download(p), _real(m, 1, n))


def _two_source_pair(n, seed, dt=0.004):
    """Two dynamic fields and an intermediate with several sources and
    operators: chi (1 + 0.3 q^2) = q^2 A + 0.2 |q|^-1 A - 0.5 i qx B,
    entering A's and B's products and a linear term of B."""
    lat = pss.Lattice(n, dt=dt, seed=seed)
    m = om.Model(_olat(n, (1.0,) * len(n)), dt, seed=seed)
    A, B, C = lat.field("A"), lat.field("B"), lat.field("chi", dynamic=False)
    Ao, Bo, Co = m.add_field("A"), m.add_field("B"), m.add_field("chi", dynamic=False)
    for side in ("gpu", "oracle"):
        M_ = Mono if side == "gpu" else OMono
        a, b, c = (A, B, C) if side == "gpu" else (Ao, Bo, Co)
        add = lat.term if side == "gpu" else (lambda t, op, fa, implicit=False: m.add_term(t, op, fa, implicit=implicit))
        add(a, [M_(-0.5), M_(-1.0, q2=1)], [(a, 1)], implicit=True)
        add(b, [M_(-0.3, q2=1), M_(-0.5, q2=2)], [(b, 1)], implicit=True)
        add(c, [M_(-0.3, q2=1)], [(c, 1)], implicit=True)
        add(c, [M_(1.0, q2=1)], [(a, 1)])
        add(c, [M_(-0.5, iq=(1, 0, 0))], [(b, 1)])
        add(c, [M_(0.2, invq=1)], [(a, 1)])
        add(a, [M_(-1.0)], [(a, 3)])
        add(a, [M_(-0.3)], [(c, 1), (a, 1)])
        add(b, [M_(0.2, q2=1)], [(c, 2)])
        add(b, [M_(-0.1)], [(c, 1)])
        add(b, [M_(-0.5, q2=1)], [(b, 3)])
    lat.noise(A, [Mono(0.004)])
    lat.noise(B, [Mono(0.004, q2=1)])
    m.set_noise(Ao, [OMono(0.004)])
    m.set_noise(Bo, [OMono(0.004, q2=1)])
    for fl in (A, B):
        lat.init_uniform(fl, -0.3, 0.3)
    for fl in (Ao, Bo):
        m.init_uniform(fl, -0.3, 0.3)
    return lat, m, (A, B, C)


@pytest.mark.parametrize("n,steps", [((64, 32), 60), ((32, 64), 60), ((16, 16, 16), 30)])
def test_intermediate_with_several_sources(n, steps):
    print(f"two-source intermediate n={n}", flush=True)
    lat, m, ids = _two_source_pair(n, seed=17)
    lat.step(steps)
    m.step(steps)
    for i, fid in enumerate(ids):
        assert _close(lat.download(fid), _real(m, i, n)), i


def test_batch_of_kpz_lattices_is_bitwise_the_single_path():
    def mk(seed):
        lat = pss.Lattice((64, 64), dx=(0.8, 0.8), dt=0.01, seed=seed)
        f, _ = pss.kpz(lat, sigma=1.0, lam=0.5, D=0.01)
        lat.init_uniform(f, -0.5, 0.5)
        return lat
    mem = [mk(s) for s in (3, 4, 5)]
    twins = [mk(s) for s in (3, 4, 5)]
    batch = pss.Batch(mem)
    batch.step(30)
    batch.sync()
    for lat, tw in zip(mem, twins):
        tw.step(30)
        assert np.array_equal(lat.spectrum(0), tw.spectrum(0))
    batch.close()
