"""Pins of the oracle's coupled two-field system and of the helpers that the
earlier pins did not reach (CPU only).

* two_field_3d (a Model B field phi coupled to a Model A field psi, the literal
  coupling reading: (g/2) phi psi^2 inside phi's chemical potential, -g phi psi
  in psi's equation):
  - at g = 0 its phi is Model B (Sec. "Example") bit for bit, noise included;
  - at g = 0 and D = 0 a uniform psi follows the scalar semi-implicit
    recursion psi <- (psi - dt psi^3) / (1 + dt c) of d/dt psi = -c psi - psi^3,
    and a faint single cosine decays as (1 + dt (c + q^2))^-n;
  - at g != 0, one step from single-cosine fields equals eq:timeupdate with
    the Fourier values of phi^3, phi psi^2, psi^3 and phi psi written from
    trigonometric product identities (no transform involved).
* adjoint.forward (the Model B run the adjoint differentiates) equals
  model_b(...).step with the same seed, noise included.
* free_energy of A cos(q x) is N dV (a A^2/4 + 3 b A^4/32 + k q^2 A^2/4).
"""

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import model as om
from oracle import observables as ob
from oracle.spectral import Lattice, fftn

DT = 0.005


def _cos_field(lat, axis, k, amp):
    n = (lat.nx, lat.ny, lat.nz)[axis]
    i = np.arange(n)
    v = amp * np.cos(2 * np.pi * k * i / n)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    return np.broadcast_to(v.reshape(shape), lat.shape).astype(np.float64)


@pytest.mark.parametrize("D", [0.0, 0.005])
def test_two_field_at_zero_coupling_is_model_b_for_phi(D):
    lat = Lattice(16, 8, 8)
    m2 = om.two_field_3d(lat, DT, g=0.0, D=D, seed=7)
    m2.init_uniform(0, -0.1, 0.1)
    m2.init_uniform(1, -0.1, 0.1)
    mb = om.model_b(lat, DT, a=-1.0, b=1.0, k=1.0, D=D, seed=7)
    mb.init_uniform(0, -0.1, 0.1)
    m2.step(15)
    mb.step(15)
    assert np.max(np.abs(m2.state[0] - mb.state[0])) <= 1e-13 * np.max(np.abs(mb.state[0]))


def test_two_field_uniform_psi_follows_the_scalar_recursion():
    lat = Lattice(8, 8, 8)
    c = -0.5
    m = om.two_field_3d(lat, DT, c=c, g=0.0, D=0.0)
    psi0 = 0.37
    m.set_real(1, np.full(lat.shape, psi0))
    m.step(40)
    want = psi0
    for _ in range(40):
        want = (want - DT * want ** 3) / (1 + DT * c)
    got = m.real(1)
    assert np.max(np.abs(got - want)) <= 1e-13
    # the opposite sign of c (or of the cube) would give a different value
    assert abs(want - psi0 * (1 - DT * c) ** 40) > 1e-3


def test_two_field_faint_psi_cosine_decays_with_c_plus_q2():
    lat = Lattice(8, 16, 8, dy=0.7)
    c, k0, amp = -0.5, 3, 1e-9
    m = om.two_field_3d(lat, DT, c=c, g=0.0, D=0.0)
    m.set_real(1, _cos_field(lat, 1, k0, amp))
    n = 60
    m.step(n)
    q = 2 * np.pi * k0 / (16 * 0.7)
    want = _cos_field(lat, 1, k0, amp) * (1 + DT * (c + q * q)) ** (-n)
    # psi^3 ~ 1e-27 is far below the 1e-15 relative tolerance
    assert np.max(np.abs(m.real(1) - want)) <= 1e-12 * amp


def test_two_field_coupling_terms_on_single_cosines():
    # phi = A cos(2 pi k1 x / Nx), psi = B cos(2 pi k2 y / Ny) on a 16^3 lattice:
    # every factor mode (|k| <= 2) is kept by the 2/3 mask and every product
    # mode (|k| <= 6 < 8) is below the Nyquist index, so the pseudo-spectral
    # products equal the exact ones.
    n = 16
    lat = Lattice(n, n, n)
    a, b, kk, c, g = -1.0, 1.0, 1.0, -0.5, 0.3
    A, B, k1, k2 = 0.4, 0.3, 1, 2
    m = om.two_field_3d(lat, DT, a=a, b=b, k=kk, c=c, g=g, D=0.0)
    m.set_real(0, _cos_field(lat, 0, k1, A))
    m.set_real(1, _cos_field(lat, 1, k2, B))
    m.step(1)

    N = lat.N

    def modes(entries):
        """Spectrum with value v*N at each listed signed (kx, ky, kz)."""
        s = np.zeros(lat.shape, dtype=complex)
        for (kx, ky, kz), v in entries:
            s[kz % n, ky % n, kx % n] += v * N
        return s
    # cos^3 t = 3/4 cos t + 1/4 cos 3t; cos t = (e^it + e^-it)/2
    def cos_modes(axis, k, amp):
        e = []
        for sgn in (1, -1):
            kv = [0, 0, 0]
            kv[axis] = sgn * k
            e.append((tuple(kv), amp / 2))
        return e
    phi0 = modes(cos_modes(0, k1, A))
    psi0 = modes(cos_modes(1, k2, B))
    phi3 = modes(cos_modes(0, k1, 0.75 * A ** 3) + cos_modes(0, 3 * k1, 0.25 * A ** 3))
    psi3 = modes(cos_modes(1, k2, 0.75 * B ** 3) + cos_modes(1, 3 * k2, 0.25 * B ** 3))
    # phi psi^2 = A B^2 cos(x) (1 + cos 2y) / 2
    phipsi2 = modes(cos_modes(0, k1, A * B * B / 2)
                    + [((sx * k1, sy * 2 * k2, 0), A * B * B / 8) for sx in (1, -1) for sy in (1, -1)])
    # phi psi = A B cos(x) cos(y) = A B / 4 sum over the four sign pairs
    phipsi = modes([((sx * k1, sy * k2, 0), A * B / 4) for sx in (1, -1) for sy in (1, -1)])
    q2 = lat.q2
    want_phi = (phi0 + DT * (-b * q2 * phi3 - 0.5 * g * q2 * phipsi2)) / (1 + DT * q2 * (a + kk * q2))
    want_psi = (psi0 + DT * (-psi3 - g * phipsi)) / (1 + DT * (c + q2))
    tol = 1e-12 * N
    assert np.max(np.abs(m.state[0] - want_phi)) <= tol
    assert np.max(np.abs(m.state[1] - want_psi)) <= tol
    # the coupling terms are not negligible at this tolerance
    assert np.max(np.abs(DT * 0.5 * g * q2 * phipsi2)) > 1e3 * tol
    assert np.max(np.abs(DT * g * phipsi)) > 1e3 * tol


@pytest.mark.parametrize("D", [0.0, 0.01])
def test_adjoint_forward_equals_model_step(D):
    lat = Lattice(32, 16)
    theta = (-0.9, 1.1, 0.9, D)
    m = om.model_b(lat, 0.01, a=theta[0], b=theta[1], k=theta[2], D=D, seed=5)
    x0 = m.init_uniform(0, -0.1, 0.1)
    mask = m._prepare()["masks"][0]
    phi0 = fftn(x0.astype(np.complex128))
    phiT, hist = adj.forward(lat, phi0, theta, 0.01, 25, 5, mask)
    m.step(25)
    scale = np.max(np.abs(m.state[0]))
    assert np.max(np.abs(phiT - m.state[0])) <= 1e-13 * scale
    # every stored state is the model's state at that step
    r = om.model_b(lat, 0.01, a=theta[0], b=theta[1], k=theta[2], D=D, seed=5)
    r.init_uniform(0, -0.1, 0.1)
    for n in (0, 1, 12, 25):
        r2 = r.copy()
        r2.step(n)
        assert np.max(np.abs(hist[n] - r2.state[0])) <= 1e-13 * scale


@pytest.mark.parametrize("k0,axis", [(3, 0), (5, 1)])
def test_free_energy_of_a_single_cosine(k0, axis):
    lat = Lattice(32, 24, 1, dx=0.5, dy=0.8)
    a, b, kk, A = -1.3, 0.7, 2.1, 0.6
    phi = _cos_field(lat, axis, k0, A)
    q = 2 * np.pi * k0 / ((32 * 0.5) if axis == 0 else (24 * 0.8))
    want = lat.N * lat.dV * (a * A ** 2 / 4 + 3 * b * A ** 4 / 32 + kk * q * q * A ** 2 / 4)
    got = ob.free_energy(lat, fftn(phi + 0j), a, b, kk)
    assert abs(got - want) <= 1e-12 * abs(want)
