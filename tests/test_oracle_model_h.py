"""Pins of the Model H oracle (oracle/model.py model_h; the paper's second
benchmark, Sec. "Benchmarking", written from Hohenberg and Halperin's model H
in the form the library takes).  Each test checks the oracle against
something other than itself:

* the projected stress operators annihilate the divergence (the pressure's
  Poisson equation), on every mode off the Nyquist planes, where the odd
  derivative i q_i is 0 by the library's convention;
* one step from rest gives the flow dt P(q) F[-phi grad mu] / (1 + dt eta q^2),
  with -phi grad mu formed independently in real space from the full
  chemical potential (a, b and k terms) and projected with real q vectors:
  the stress form, its sign, the factor 2 of the mixed product and the
  cancellation of the a and b parts are all pinned by it;
* an advected single mode follows the closed form of one step;
* a profile that depends on x only drives no flow and follows the Model B
  oracle exactly;
* the mean of phi is conserved and the flow stays solenoidal under noise;
* with no noise the free energy plus the kinetic energy does not grow;
* in 3D: the same projection, one-step, flat-profile and invariant checks.
"""

import numpy as np

from oracle import model as om
from oracle import observables as ob
from oracle.spectral import Lattice, fftn, ifftn


def _off_nyquist(lat):
    keep = np.ones(lat.shape, dtype=bool)
    for i, n in enumerate((lat.nx, lat.ny)):
        keep &= lat.k_int[i] != -(n // 2)
    return keep


def test_projected_stress_is_solenoidal():
    lat = Lattice(32, 16, dx=0.7, dy=1.3)
    ops = om.model_h_force_ops(1.7)
    keep = _off_nyquist(lat) & (lat.q2 > 0)
    for ij in ((0, 0), (0, 1), (1, 1)):
        ox = lat.operator(ops[(0, ij)])
        oy = lat.operator(ops[(1, ij)])
        div = lat.iq[0] * ox + lat.iq[1] * oy
        scale = np.max(np.abs(lat.iq[0] * ox))
        assert scale > 1.0
        assert np.max(np.abs(div[keep])) <= 1e-12 * scale, ij


def _smooth(lat, rng, kmax):
    """A real field with random modes |k_i| <= kmax only."""
    spec = np.zeros(lat.shape, dtype=np.complex128)
    sel = (np.abs(lat.k_int[0]) <= kmax) & (np.abs(lat.k_int[1]) <= kmax)
    sel = np.broadcast_to(sel, lat.shape)
    spec[sel] = rng.normal(size=sel.sum()) + 1j * rng.normal(size=sel.sum())
    x = ifftn(spec).real
    return 0.6 * x / np.max(np.abs(x))


def test_one_step_flow_is_the_projected_phi_grad_mu():
    n, dt = 64, 0.02
    a, b, k, M, eta = -0.8, 1.3, 0.9, 0.7, 1.6
    lat = Lattice(n, n, dx=0.9, dy=0.9)
    rng = np.random.default_rng(4)
    phi0 = _smooth(lat, rng, 4)  # products stay far below the de-aliasing cutoff
    m = om.model_h(lat, dt, a=a, b=b, k=k, M=M, eta=eta, D=0.0)
    m.set_real(0, phi0)
    m.step(1)
    # independent: f = -phi grad mu in real space, projected with real q
    ph = fftn(phi0.astype(np.complex128))
    mu = a * phi0 + b * phi0 ** 3 + k * ifftn(lat.q2 * ph).real  # -k lap phi = k F^-1[q^2 phi]
    muh = fftn(mu.astype(np.complex128))
    q = [np.broadcast_to(lat.q[i], lat.shape) for i in range(2)]
    f = [fftn((-phi0 * ifftn(1j * q[i] * muh).real).astype(np.complex128)) for i in range(2)]
    with np.errstate(divide="ignore", invalid="ignore"):
        qf = (q[0] * f[0] + q[1] * f[1]) / np.where(lat.q2 > 0, lat.q2, 1.0)
    pf = [np.where(lat.q2 > 0, f[i] - q[i] * qf, 0.0) for i in range(2)]
    for i in range(2):
        want = dt * pf[i] / (1.0 + dt * eta * lat.q2)
        got = m.state[1 + i]
        assert np.max(np.abs(want)) > 1e-3
        assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want)), i
    # phi: a Model B step (the flow starts at rest)
    mb = om.model_b(lat, dt, a=M * a, b=M * b, k=M * k, D=0.0)
    mb.set_real(0, phi0)
    mb.step(1)
    assert np.max(np.abs(m.state[0] - mb.state[0])) <= 1e-12 * np.max(np.abs(mb.state[0]))


def test_advected_mode_closed_form():
    n, dt, U, eta = 32, 0.05, 0.8, 0.3
    L = n * 1.0
    lat = Lattice(n, n)
    m = om.model_h(lat, dt, a=0.0, b=0.0, k=0.0, M=1.0, eta=eta, D=0.0)
    q1 = 2 * np.pi / L
    x = np.arange(n)[None, None, :] * 1.0
    y = np.arange(n)[None, :, None] * 1.0
    phi0 = np.broadcast_to(np.cos(q1 * x), lat.shape)
    vx0 = np.broadcast_to(U * np.sin(q1 * y), lat.shape)
    m.set_real(0, phi0)
    m.set_real(1, vx0)
    m.step(1)
    want_phi = np.cos(q1 * x) + dt * U * q1 * np.sin(q1 * y) * np.sin(q1 * x)
    assert np.max(np.abs(m.real(0) - want_phi)) <= 1e-12
    assert np.max(np.abs(m.real(1) - vx0 / (1.0 + dt * eta * q1 ** 2))) <= 1e-12
    assert np.max(np.abs(m.real(2))) <= 1e-14


def test_flat_profile_drives_no_flow_and_follows_model_b():
    n, dt = 64, 0.01
    lat = Lattice(n, 16)
    rng = np.random.default_rng(2)
    prof = rng.uniform(-0.5, 0.5, size=n)
    phi0 = np.broadcast_to(prof[None, None, :], lat.shape)
    m = om.model_h(lat, dt, D=0.0)
    mb = om.model_b(lat, dt, D=0.0)
    m.set_real(0, phi0)
    mb.set_real(0, phi0)
    m.step(50)
    mb.step(50)
    assert np.max(np.abs(m.real(1))) <= 1e-13
    assert np.max(np.abs(m.real(2))) <= 1e-13
    assert np.max(np.abs(m.real(0) - mb.real(0))) <= 1e-12


def test_mass_is_conserved_and_the_flow_stays_solenoidal():
    lat = Lattice(32, 64, dx=0.8, dy=0.8)
    m = om.model_h(lat, 0.01, D=0.02, seed=9)
    m.init_uniform(0, -0.4, 0.6)
    mass0 = m.state[0][0, 0, 0].real
    m.step(60)
    assert abs(m.state[0][0, 0, 0].real - mass0) <= 1e-10 * np.sum(np.abs(m.real(0)))
    keep = _off_nyquist(lat)
    div = lat.iq[0] * m.state[1] + lat.iq[1] * m.state[2]
    vmax = np.max(np.sqrt(lat.q2) * (np.abs(m.state[1]) + np.abs(m.state[2])))
    assert vmax > 0
    assert np.max(np.abs(div[keep])) <= 1e-12 * vmax


def test_energy_does_not_grow_without_noise():
    a, b, k = -1.0, 1.0, 1.0
    lat = Lattice(32, 32)
    m = om.model_h(lat, 0.01, a=a, b=b, k=k, D=0.0, seed=5)
    m.init_uniform(0, -0.3, 0.3)
    prev = None
    for _ in range(40):
        m.step(5)
        s = m.spectra()
        kin = 0.5 * lat.dV * np.sum(m.real(1) ** 2 + m.real(2) ** 2)
        e = ob.free_energy(lat, s[0], a, b, k) + kin
        if prev is not None:
            assert e <= prev + 1e-12 * abs(prev)
        prev = e


# -- three dimensions ---------------------------------------------------------

def _off_nyquist3(lat):
    keep = np.ones(lat.shape, dtype=bool)
    for i, n in enumerate((lat.nx, lat.ny, lat.nz)):
        keep &= lat.k_int[i] != -(n // 2)
    return keep


def test_projected_stress_is_solenoidal_3d():
    lat = Lattice(16, 8, 12, dx=0.7, dy=1.3, dz=0.9)
    ops = om.model_h_force_ops(1.3, ndim=3)
    assert len(ops) == 18
    keep = _off_nyquist3(lat) & (lat.q2 > 0)
    for i in range(3):
        for j in range(i, 3):
            div = sum(lat.iq[c] * lat.operator(ops[(c, (i, j))]) for c in range(3))
            scale = max(np.max(np.abs(lat.iq[c] * lat.operator(ops[(c, (i, j))]))) for c in range(3))
            assert scale > 1.0
            assert np.max(np.abs(div[keep])) <= 1e-12 * scale, (i, j)


def test_one_step_flow_is_the_projected_phi_grad_mu_3d():
    n, dt = 16, 0.02
    a, b, k, M, eta = -0.7, 1.2, 0.8, 0.9, 1.4
    lat = Lattice(n, n, n, dx=0.8, dy=0.8, dz=0.8)
    rng = np.random.default_rng(8)
    spec = np.zeros(lat.shape, dtype=np.complex128)
    sel = np.broadcast_to((np.abs(lat.k_int[0]) <= 1) & (np.abs(lat.k_int[1]) <= 1) & (np.abs(lat.k_int[2]) <= 1),
                          lat.shape)
    spec[sel] = rng.normal(size=sel.sum()) + 1j * rng.normal(size=sel.sum())
    phi0 = ifftn(spec).real
    phi0 = 0.6 * phi0 / np.max(np.abs(phi0))
    m = om.model_h(lat, dt, a=a, b=b, k=k, M=M, eta=eta, D=0.0)
    m.set_real(0, phi0)
    m.step(1)
    ph = fftn(phi0.astype(np.complex128))
    mu = a * phi0 + b * phi0 ** 3 + k * ifftn(lat.q2 * ph).real
    muh = fftn(mu.astype(np.complex128))
    q = [np.broadcast_to(lat.q[i], lat.shape) for i in range(3)]
    f = [fftn((-phi0 * ifftn(1j * q[i] * muh).real).astype(np.complex128)) for i in range(3)]
    qf = sum(q[i] * f[i] for i in range(3)) / np.where(lat.q2 > 0, lat.q2, 1.0)
    for i in range(3):
        want = dt * np.where(lat.q2 > 0, f[i] - q[i] * qf, 0.0) / (1.0 + dt * eta * lat.q2)
        got = m.state[1 + i]
        assert np.max(np.abs(want)) > 1e-4
        assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want)), i


def test_flat_profile_drives_no_flow_3d():
    lat = Lattice(32, 8, 8)
    prof = np.random.default_rng(3).uniform(-0.5, 0.5, size=32)
    m = om.model_h(lat, 0.01, D=0.0)
    mb = om.model_b(lat, 0.01, D=0.0)
    phi0 = np.broadcast_to(prof[None, None, :], lat.shape)
    m.set_real(0, phi0)
    mb.set_real(0, phi0)
    m.step(30)
    mb.step(30)
    for c in (1, 2, 3):
        assert np.max(np.abs(m.real(c))) <= 1e-13
    assert np.max(np.abs(m.real(0) - mb.real(0))) <= 1e-12


def test_mass_and_divergence_3d():
    lat = Lattice(16, 16, 8)
    m = om.model_h(lat, 0.01, D=0.02, seed=4)
    m.init_uniform(0, -0.4, 0.5)
    mass0 = m.state[0][0, 0, 0].real
    m.step(30)
    assert abs(m.state[0][0, 0, 0].real - mass0) <= 1e-10 * np.sum(np.abs(m.real(0)))
    div = sum(lat.iq[c] * m.state[1 + c] for c in range(3))
    vmax = np.max(np.sqrt(lat.q2) * sum(np.abs(m.state[1 + c]) for c in range(3)))
    assert vmax > 0
    assert np.max(np.abs(div[_off_nyquist3(lat)])) <= 1e-12 * vmax
