"""Pins of the oracle's boundary frames (Sec. "Callback functions": a field
held at fixed values on a band of sites at the end of every step), CPU only.

* A frame whose values equal the field changes nothing.
* Without dynamics (no terms) one step leaves the frame values on the frame
  sites and every other site untouched.
* One diffusion step from a uniform field is still uniform before the frame,
  so afterwards the field is the frame on its sites and the uniform value
  elsewhere.
* The paper's heat-bath example: 1D diffusion between a band of sites held
  at T1 and one held at T2 (frames of width 10 on 256 sites, T(x, 0) = 5)
  relaxes to the straight line between the two baths across the interior
  (within 2% of T1 - T2 after a long run); a single-site frame leaves the
  periodic artefact, a steady state far from that line.
"""

import numpy as np

from oracle import model as om
from oracle.spectral import Lattice, Mono


def _diffusion(n, dt, D=1.0):
    m = om.Model(Lattice(n), dt)
    f = m.add_field("T")
    m.add_term(f, [Mono(-D, q2=1)], [(f, 1)], implicit=True)
    return m


def test_frame_equal_to_the_field_changes_nothing():
    lat = Lattice(16, 8)
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    rng = np.random.default_rng(1)
    x = rng.normal(size=lat.shape)
    m.set_real(f, x)
    sites = np.array([0, 5, 17, 100])
    m.set_frame(f, sites, x.reshape(-1)[sites])
    m.step(3)
    assert np.max(np.abs(m.real(f) - x)) <= 1e-13


def test_frame_without_dynamics():
    lat = Lattice(32)
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    x = np.sin(np.arange(32) * 0.3).reshape(lat.shape)
    m.set_real(f, x)
    m.set_frame(f, [0, 1, 31], [2.0, -1.0, 0.5])
    m.step(1)
    want = x.reshape(-1).copy()
    want[[0, 1, 31]] = [2.0, -1.0, 0.5]
    assert np.max(np.abs(m.real(f).reshape(-1) - want)) <= 1e-13


def test_one_diffusion_step_from_uniform():
    m = _diffusion(64, 0.1)
    m.set_real(0, np.full(m.lat.shape, 5.0))
    sites = list(range(10)) + list(range(54, 64))
    m.set_frame(0, sites, [10.0] * 10 + [0.0] * 10)
    m.step(1)
    want = np.full(64, 5.0)
    want[:10] = 10.0
    want[54:] = 0.0
    assert np.max(np.abs(m.real(0).reshape(-1) - want)) <= 1e-12


def test_heat_baths_relax_to_the_straight_line():
    n, w, T1, T2 = 256, 10, 10.0, 0.0
    m = _diffusion(n, 1.0)
    m.set_real(0, np.full(m.lat.shape, 5.0))
    sites = list(range(w)) + list(range(n - w, n))
    m.set_frame(0, sites, [T1] * w + [T2] * w)
    m.step(20000)
    x = np.arange(n)
    inner = slice(w, n - w)
    line = T1 + (T2 - T1) * (x - (w - 1)) / ((n - w) - (w - 1))
    err = np.max(np.abs(m.real(0).reshape(-1)[inner] - line[inner]))
    assert err <= 0.02 * abs(T1 - T2), err
    # a one-site bath at each end: the periodic jump T2 -> T1 across the
    # boundary keeps the profile far from the line
    m1 = _diffusion(n, 1.0)
    m1.set_real(0, np.full(m1.lat.shape, 5.0))
    m1.set_frame(0, [0, n - 1], [T1, T2])
    m1.step(20000)
    err1 = np.max(np.abs(m1.real(0).reshape(-1)[1:n - 1] - (T1 + (T2 - T1) * (x[1:n - 1]) / (n - 1))))
    assert err1 >= 0.1 * abs(T1 - T2), err1
