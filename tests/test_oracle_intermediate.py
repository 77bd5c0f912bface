"""Pins of the oracle's intermediate (non-dynamic) fields and of the KPZ model
built from them (CPU only).

Every expected value below is written in real space from trigonometric
identities and the wave numbers q = 2 pi k / (N dx); no transform is involved.

* The paper's intermediate example (Sec. "Writing models"):
  psi + psi q^2 = -q^2 phi, i.e. psi_hat = -q^2 (1 + q^2)^-1 phi_hat, on a
  sum of two cosines of different |q| and non-unit spacings.
* psi = i q_x phi is the x derivative of phi; on the Nyquist column it is zero
  (i q_i vanishes on the Nyquist plane of axis i).
* One KPZ step (Sec. "What cuPSS calculates") from A cos(q_x x) + B cos(q_y y)
  without noise: the nonlinearity lam ((d_x phi)^2 + (d_y phi)^2) has modes 0,
  2 q_x and 2 q_y, each divided by 1 + dt sigma q^2 (eq:timeupdate); a mode
  above the 2/3 cutoff of the squared gradients contributes no nonlinearity.
* An intermediate whose right-hand side is a product (c = phi^3) used in a
  linear term (d/dt phi = -b q^2 c) reproduces Model B (Sec. "Example") to
  rounding, noise included: the de-aliasing order of phi comes from the
  intermediate's product.
* A linear intermediate with a denominator inside a linear term gives the
  closed-form per-mode recursion over several steps.
* Misuse is refused: noise on an intermediate, an intermediate that uses a
  later one, a singular intermediate equation.
"""

import numpy as np
import pytest

from oracle import model as om
from oracle.spectral import Lattice, Mono


def _coords(lat):
    z, y, x = np.meshgrid(np.arange(lat.nz) * lat.dz, np.arange(lat.ny) * lat.dy, np.arange(lat.nx) * lat.dx,
                          indexing="ij")
    return x, y, z


def _wave(n, d, k):
    return 2 * np.pi * k / (n * d)


def test_paper_intermediate_closed_form():
    lat = Lattice(32, 16, dx=0.7, dy=1.3)
    x, y, _ = _coords(lat)
    qa = (_wave(32, 0.7, 3), _wave(16, 1.3, 2))
    qb = (_wave(32, 0.7, 7), 0.0)
    phi = 0.8 * np.cos(qa[0] * x + qa[1] * y) + 0.3 * np.sin(qb[0] * x)
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    psi = m.add_field("psi", dynamic=False)
    # psi + psi q^2 = -q^2 phi: the implicit part -q^2 on the right-hand side
    m.add_term(psi, [Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    m.add_term(psi, [Mono(-1.0, q2=1)], [(f, 1)])
    m.set_real(f, phi)
    q2a = qa[0] ** 2 + qa[1] ** 2
    q2b = qb[0] ** 2
    want = -q2a / (1 + q2a) * 0.8 * np.cos(qa[0] * x + qa[1] * y) - q2b / (1 + q2b) * 0.3 * np.sin(qb[0] * x)
    assert np.max(np.abs(m.real(psi) - want)) <= 1e-13
    # the dynamic field is unchanged by reading the intermediate
    assert np.max(np.abs(m.real(f) - phi)) <= 1e-13


def test_gradient_intermediate_and_nyquist():
    lat = Lattice(16, 8, dx=0.5, dy=2.0)
    x, y, _ = _coords(lat)
    qx, qy = _wave(16, 0.5, 3), _wave(8, 2.0, 1)
    phi = 0.6 * np.cos(qx * x + qy * y) + 0.2 * np.cos(np.pi * x / 0.5)  # second term: Nyquist column
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    gx = m.add_field("gx", dynamic=False)
    gy = m.add_field("gy", dynamic=False)
    m.add_term(gx, [Mono(1.0, iq=(1, 0, 0))], [(f, 1)])
    m.add_term(gy, [Mono(1.0, iq=(0, 1, 0))], [(f, 1)])
    m.set_real(f, phi)
    assert np.max(np.abs(m.real(gx) - (-0.6 * qx * np.sin(qx * x + qy * y)))) <= 1e-13
    assert np.max(np.abs(m.real(gy) - (-0.6 * qy * np.sin(qx * x + qy * y)))) <= 1e-13


@pytest.mark.parametrize("kx,ky", [(2, 3), (11, 3)])
def test_kpz_first_step_closed_form(kx, ky):
    n, dx, dt, sigma, lam = 32, 0.9, 0.02, 1.3, 0.7
    lat = Lattice(n, n, dx=dx, dy=dx)
    x, y, _ = _coords(lat)
    qx, qy = _wave(n, dx, kx), _wave(n, dx, ky)
    A, B = 0.4, 0.25
    m = om.kpz(lat, dt, sigma=sigma, lam=lam, D=0.0)
    m.set_real(0, A * np.cos(qx * x) + B * np.cos(qy * y))
    m.step(1)

    def keep(k1, k2):  # 2/3 radial cutoff of the squared gradients (order 2)
        return (k1 / (n / 2)) ** 2 + (k2 / (n / 2)) ** 2 < (2 / 3) ** 2
    # lam (d_x phi)^2 = lam A^2 qx^2 sin^2(qx x) = lam A^2 qx^2 (1 - cos(2 qx x)) / 2
    ax = lam * A * A * qx * qx / 2 if keep(kx, 0) else 0.0
    ay = lam * B * B * qy * qy / 2 if keep(0, ky) else 0.0
    want = (A * np.cos(qx * x) / (1 + dt * sigma * qx * qx) + B * np.cos(qy * y) / (1 + dt * sigma * qy * qy)
            + dt * (ax + ay)
            - dt * ax * np.cos(2 * qx * x) / (1 + dt * sigma * 4 * qx * qx)
            - dt * ay * np.cos(2 * qy * y) / (1 + dt * sigma * 4 * qy * qy))
    assert np.max(np.abs(m.real(0) - want)) <= 1e-13


@pytest.mark.parametrize("D", [0.0, 0.01])
def test_product_intermediate_reproduces_model_b(D):
    lat = Lattice(32, 16)
    a, b, k, dt = -1.0, 1.0, 1.0, 0.01
    mb = om.model_b(lat, dt, a=a, b=b, k=k, D=D, seed=5)
    mb.init_uniform(0, -0.3, 0.3)
    m = om.Model(lat, dt, seed=5)
    f = m.add_field("phi")
    c = m.add_field("cube", dynamic=False)
    m.add_term(f, [Mono(-a, q2=1), Mono(-k, q2=2)], [(f, 1)], implicit=True)
    m.add_term(c, [Mono(1.0)], [(f, 3)])
    m.add_term(f, [Mono(-b, q2=1)], [(c, 1)])
    if D:
        m.set_noise(f, [Mono(D, q2=1)])
    m.init_uniform(0, -0.3, 0.3)
    mb.step(25)
    m.step(25)
    assert np.max(np.abs(m.state[0] - mb.state[0])) <= 1e-12 * np.max(np.abs(mb.state[0]))


def test_rational_intermediate_in_a_linear_term():
    lat = Lattice(16, 16, dx=1.1, dy=1.1)
    x, y, _ = _coords(lat)
    qx, qy = _wave(16, 1.1, 2), _wave(16, 1.1, 5)
    dt, steps = 0.05, 12
    m = om.Model(lat, dt)
    f = m.add_field("phi")
    psi = m.add_field("psi", dynamic=False)
    m.add_term(f, [Mono(-0.5, q2=1)], [(f, 1)], implicit=True)          # L = -0.5 q^2
    m.add_term(psi, [Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)      # psi + q^2 psi = -q^2 phi
    m.add_term(psi, [Mono(-1.0, q2=1)], [(f, 1)])
    m.add_term(f, [Mono(-0.8)], [(psi, 1)])                           # d/dt phi += -0.8 psi
    m.set_real(f, np.cos(qx * x) + 0.5 * np.sin(qy * y))
    m.step(steps)

    def gain(q2):
        return (1 + dt * 0.8 * q2 / (1 + q2)) / (1 + dt * 0.5 * q2)
    want = gain(qx * qx) ** steps * np.cos(qx * x) + 0.5 * gain(qy * qy) ** steps * np.sin(qy * y)
    assert np.max(np.abs(m.real(f) - want)) <= 1e-13


def test_intermediate_misuse_is_refused():
    lat = Lattice(8, 8)
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    g = m.add_field("g", dynamic=False)
    with pytest.raises(ValueError):
        m.set_noise(g, [Mono(1.0)])
    with pytest.raises(ValueError):
        m.set_real(g, np.zeros(lat.shape))
    # g uses h, declared after it
    h = m.add_field("h", dynamic=False)
    m.add_term(h, [Mono(1.0)], [(f, 1)])
    m.add_term(g, [Mono(1.0)], [(h, 2)])
    m.add_term(f, [Mono(1.0)], [(g, 1)])
    with pytest.raises(ValueError):
        m.step(1)
    # psi = psi + phi has no solution: 1 - L_psi = 0 everywhere
    m2 = om.Model(lat, 0.01)
    f2 = m2.add_field("phi")
    p2 = m2.add_field("psi", dynamic=False)
    m2.add_term(p2, [Mono(1.0)], [(p2, 1)], implicit=True)
    m2.add_term(p2, [Mono(1.0)], [(f2, 1)])
    with pytest.raises(ValueError):
        m2.step(1)
