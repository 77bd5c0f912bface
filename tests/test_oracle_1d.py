"""Pins of the oracle on 1D lattices (CPU only), the dimension of the paper's
examples in Sec. "De-aliasing" and Sec. "Callback functions".

Every expected value is written in real space from trigonometric identities
and q = 2 pi k / (N dx); no transform is involved.

* Diffusion d/dt phi = D lap phi: each cosine decays as (1 + dt D q^2)^-n
  (eq:timeupdate with the implicit operator -D q^2).
* One Model B step (Sec. "Example") from A cos(q x): the cube is
  A^3 (3 cos(q x) + cos(3 q x)) / 4.  The 2/3 cutoff masks the factor, not
  its cube, so both harmonics are present whenever q itself is kept (3q
  folding back onto the lattice when it passes Nyquist), and none when q is
  cut.
* One KPZ step from A cos(q x): (d_x phi)^2 = A^2 q^2 (1 - cos(2 q x)) / 2.
* Conserved noise (D q^2) leaves the mean untouched; non-conserved noise
  moves it as a random walk of variance 2 D dt n / (N dx).
"""

import numpy as np
import pytest

from oracle import model as om
from oracle.spectral import Lattice, Mono


def _x(lat):
    return np.arange(lat.nx) * lat.dx


def test_diffusion_decay_closed_form():
    n, dx, dt, D, steps = 64, 0.7, 0.05, 0.9, 30
    lat = Lattice(n, dx=dx)
    x = _x(lat)
    m = om.Model(lat, dt)
    f = m.add_field("phi")
    m.add_term(f, [Mono(-D, q2=1)], [(f, 1)], implicit=True)
    q1, q2 = 2 * np.pi * 3 / (n * dx), 2 * np.pi * 11 / (n * dx)
    m.set_real(f, np.cos(q1 * x) + 0.4 * np.sin(q2 * x))
    m.step(steps)
    want = (1 + dt * D * q1 * q1) ** -steps * np.cos(q1 * x) + 0.4 * (1 + dt * D * q2 * q2) ** -steps * np.sin(q2 * x)
    assert np.max(np.abs(m.real(f)[0, 0] - want)) <= 1e-13


@pytest.mark.parametrize("k", [2, 9, 11])
def test_model_b_first_step_closed_form(k):
    n, dx, dt, a, b, kk, A = 32, 1.0, 0.01, -1.0, 1.0, 1.0, 0.3
    lat = Lattice(n, dx=dx)
    x = _x(lat)
    m = om.model_b(lat, dt, a=a, b=b, k=kk, D=0.0)
    q = 2 * np.pi * k / (n * dx)
    m.set_real(0, A * np.cos(q * x))
    m.step(1)
    kept = (k / (n / 2)) ** 2 < (2 / 3) ** 2  # 2/3 cutoff of the factor (radial = |k| in 1D)

    def lam(qq):
        return qq * qq * (a + kk * qq * qq)
    c1 = A - (dt * b * q * q * 0.75 * A ** 3 if kept else 0.0)
    want = c1 / (1 + dt * lam(q)) * np.cos(q * x)
    if kept:
        q3 = 3 * q
        k3 = (3 * k) % n
        k3 = k3 if k3 <= n // 2 else k3 - n  # the harmonic 3k folds back on the lattice
        q3 = 2 * np.pi * k3 / (n * dx)
        want = want - dt * b * q3 * q3 * 0.25 * A ** 3 / (1 + dt * lam(q3)) * np.cos(q3 * x)
    assert np.max(np.abs(m.real(0)[0, 0] - want)) <= 1e-13


def test_kpz_first_step_closed_form():
    n, dx, dt, sigma, lamda, A, k = 64, 0.8, 0.02, 1.3, 0.7, 0.4, 5
    lat = Lattice(n, dx=dx)
    x = _x(lat)
    m = om.kpz(lat, dt, sigma=sigma, lam=lamda, D=0.0)
    assert m.names == ["phi", "dx_phi"]  # one gradient intermediate in 1D
    q = 2 * np.pi * k / (n * dx)
    m.set_real(0, A * np.cos(q * x))
    m.step(1)
    a0 = lamda * A * A * q * q / 2
    want = (A * np.cos(q * x) / (1 + dt * sigma * q * q) + dt * a0
            - dt * a0 * np.cos(2 * q * x) / (1 + dt * sigma * 4 * q * q))
    assert np.max(np.abs(m.real(0)[0, 0] - want)) <= 1e-13


def test_noise_mean_in_1d():
    n, dx, dt, D, steps = 64, 0.5, 0.01, 0.3, 100
    # conserved noise: the mean (mode 0) never moves
    lat = Lattice(n, dx=dx)
    m = om.Model(lat, dt, seed=3)
    f = m.add_field("phi")
    m.set_noise(f, [Mono(D, q2=1)])
    m.step(50)
    assert abs(m.state[0][0, 0, 0]) <= 1e-12
    # non-conserved noise: the mean is a random walk, variance 2 D dt n / (N dx)
    means = []
    for seed in range(200):
        m = om.Model(lat, dt, seed=seed)
        f = m.add_field("phi")
        m.set_noise(f, [Mono(D)])
        m.step(steps)
        means.append(m.state[0][0, 0, 0].real / n)
    var = np.var(means)
    want = 2 * D * dt * steps / (n * dx)
    # 200 samples: the sample variance is within 30% of the truth (4.2 sigma)
    assert abs(var - want) <= 0.3 * want
