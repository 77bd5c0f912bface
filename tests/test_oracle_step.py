"""Pins of the oracle's time step against closed forms and exact properties
of the scheme (CPU only).

* eq:timeupdate with no nonlinearity and no noise is a per-mode geometric
  sequence: phi_n = phi_0 ((1 + dt M)/(1 - dt L))^n, and for coupled fields a
  per-mode matrix power (the Jacobi reading of the six-step list).
* with noise and a linear operator the per-mode variance is a finite
  geometric series (Ornstein-Uhlenbeck in discrete time); a q = 0 mode with
  no restoring force is a random walk; conserved noise (D q^2, Sec. "Adding
  noise") leaves the q = 0 mode untouched.
* eq:cubicexample on a single cosine gives the exact triple-angle values.
* with the order rule of Sec. "De-aliasing" the retained modes of the
  pseudo-spectral product equal the exact (non-periodic) convolution.
* Model B (Sec. "Example") conserves mass exactly, keeps the stationary kink
  sqrt(-a/b) tanh(x / sqrt(2k/(-a))) and lowers its free energy.
"""

import itertools

import numpy as np
import pytest

from oracle import model as om
from oracle import observables as ob
from oracle.spectral import (Lattice, Mono, fftn, ifftn, DEALIAS_PAPER_ORDER,
                             DEALIAS_TWO_THIRDS, SHAPE_PER_AXIS, SHAPE_RADIAL)


def _rand_field(lat, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    return amp * rng.standard_normal(lat.shape)


# ---------------------------------------------------------------- linear ---
def test_implicit_decay_closed_form():
    lat = Lattice(16, 8, 1, dx=0.7, dy=1.3)
    dt = 0.05
    m = om.Model(lat, dt)
    f = m.add_field("phi")
    imp = [Mono(-0.3, q2=1), Mono(-0.1, q2=2), Mono(0.2, iq=(2, 0, 0)), Mono(-0.05, invq=1),
           Mono(0.02, iq=(0, 1, 0))]
    m.add_term(f, imp, [(f, 1)], implicit=True)
    phi0 = _rand_field(lat, 3)
    m.set_real(f, phi0)
    s0 = m.state[f].copy()
    n = 37
    m.step(n)
    # closed form, operators rebuilt from q directly
    qx, qy = lat.q[0], lat.q[1]
    iqx = np.where(lat.k_int[0] == -8, 0, qx)
    iqy = np.where(lat.k_int[1] == -4, 0, qy)
    q2 = qx ** 2 + qy ** 2
    with np.errstate(divide="ignore"):
        invq = np.where(q2 > 0, 1 / np.sqrt(np.where(q2 > 0, q2, 1)), 0)
    L = -0.3 * q2 - 0.1 * q2 ** 2 - 0.2 * iqx ** 2 - 0.05 * invq + 0.02j * iqy
    want = s0 * (1 - dt * L) ** (-n)
    assert np.max(np.abs(m.state[f] - want)) <= 1e-12 * np.max(np.abs(want))


def test_explicit_linear_and_jacobi_coupling_closed_form():
    lat = Lattice(8, 8)
    dt = 0.02
    m = om.Model(lat, dt)
    a = m.add_field("a")
    b = m.add_field("b")
    m.add_term(a, [Mono(-1.0, q2=1)], [(a, 1)], implicit=True)
    m.add_term(b, [Mono(-0.5), Mono(-2.0, q2=1)], [(b, 1)], implicit=True)
    m.add_term(a, [Mono(0.7, iq=(1, 0, 0))], [(b, 1)])       # explicit cross
    m.add_term(b, [Mono(-0.4, q2=1)], [(a, 1)])              # explicit cross
    m.add_term(a, [Mono(0.3)], [(a, 1)])                     # explicit self
    m.set_real(a, _rand_field(lat, 4))
    m.set_real(b, _rand_field(lat, 5))
    A0, B0 = m.state[a].copy(), m.state[b].copy()
    n = 25
    m.step(n)
    q2 = lat.q2
    iqx = np.where(lat.k_int[0] == -4, 0, lat.q[0]) * 1j
    iqx = np.broadcast_to(iqx, lat.shape)
    da = 1 + dt * q2
    db = 1 + dt * (0.5 + 2.0 * q2)
    # per-mode Jacobi matrix [[(1+0.3dt)/da, 0.7 iqx dt/da], [-0.4 q2 dt/db, 1/db]]
    Ma = np.stack([np.stack([(1 + 0.3 * dt) / da, 0.7 * iqx * dt / da]),
                   np.stack([-0.4 * q2 * dt / db, 1 / db + 0 * da])])
    Ma = np.moveaxis(Ma, (0, 1), (-2, -1))
    P = np.linalg.matrix_power(Ma, n)
    v0 = np.stack([A0, B0], axis=-1)[..., None]
    v = (P @ v0)[..., 0]
    assert np.max(np.abs(m.state[a] - v[..., 0])) < 1e-12 * np.max(np.abs(v))
    assert np.max(np.abs(m.state[b] - v[..., 1])) < 1e-12 * np.max(np.abs(v))


# ----------------------------------------------------------------- noise ---
@pytest.mark.parametrize("conserved", [True, False])
def test_ou_variance_from_zero(conserved):
    lat = Lattice(64, 32, 1, dx=0.5, dy=0.8)
    dt, n, D = 0.05, 60, 0.3
    lam_ops = [Mono(-0.4), Mono(-1.0, q2=1)]
    ratios = []
    for seed in range(4):
        m = om.Model(lat, dt, seed=seed)
        f = m.add_field("phi")
        m.add_term(f, lam_ops, [(f, 1)], implicit=True)
        m.set_noise(f, [Mono(D, q2=1)] if conserved else [Mono(D)])
        m.step(n)
        A = 1 + dt * (0.4 + lat.q2)
        Dq = D * lat.q2 if conserved else D + 0 * lat.q2
        var = (lat.N / lat.dV) * 2 * Dq * dt * (1 - A ** (-2 * n)) / (A ** 2 - 1)
        sel = var > 0
        ratios.append((np.abs(m.state[f]) ** 2)[sel] / var[sel])
        if conserved:
            assert m.state[f][0, 0, 0] == 0
    r = np.concatenate([x.reshape(-1) for x in ratios])
    nind = r.size / 2  # modes come in conjugate pairs
    se = 1 / np.sqrt(nind)
    assert abs(r.mean() - 1) < 4 * se
    # the q-dependence: low and high halves separately
    q2s = np.concatenate([np.broadcast_to(lat.q2, lat.shape)[
        (lat.q2 > 0) if conserved else np.ones(lat.shape, bool)].reshape(-1)] * 4)
    lo = r[q2s < np.median(q2s)]
    hi = r[q2s >= np.median(q2s)]
    assert abs(lo.mean() - 1) < 4 * np.sqrt(2 / lo.size)
    assert abs(hi.mean() - 1) < 4 * np.sqrt(2 / hi.size)


def test_stationary_ou_variance():
    # long run: per-mode variance reaches (N/dV) D(q) / (lam (1 + dt lam / 2))
    lat = Lattice(32, 32, 1, dx=1.5, dy=1.5)
    dt, D = 0.1, 0.05
    m = om.Model(lat, dt, seed=11)
    f = m.add_field("phi")
    m.add_term(f, [Mono(-1.0), Mono(-1.0, q2=1)], [(f, 1)], implicit=True)
    m.set_noise(f, [Mono(D)])
    m.step(200)  # A^-400 < 1e-16 for lam >= 1
    lam = 1.0 + lat.q2
    want = (lat.N / lat.dV) * D / (lam * (1 + dt * lam / 2))
    r = np.abs(m.state[f]) ** 2 / want
    assert abs(r.mean() - 1) < 4 * np.sqrt(2 / r.size)


def test_zero_mode_random_walk():
    lat = Lattice(4, 4, 1, dx=0.5, dy=0.5)
    dt, n, D = 0.1, 20, 0.7
    vals = []
    for seed in range(400):
        m = om.Model(lat, dt, seed=seed)
        f = m.add_field("phi")
        m.add_term(f, [Mono(-1.0, q2=1)], [(f, 1)], implicit=True)
        m.set_noise(f, [Mono(D)])
        m.step(n)
        vals.append(m.state[f][0, 0, 0])
    vals = np.array(vals)
    assert np.max(np.abs(vals.imag)) == 0
    var = n * 2 * D * dt * lat.N / lat.dV
    r = vals.real ** 2 / var
    assert abs(r.mean() - 1) < 4 * np.sqrt(2 / r.size)


def test_noise_is_hermitian_and_keyed():
    lat = Lattice(8, 6, 4)
    m = om.Model(lat, 0.1, seed=5)
    f = m.add_field("phi")
    xi = m.noise_hat(f, 3)
    flip = xi[(-np.arange(4)) % 4][:, (-np.arange(6)) % 6][:, :, (-np.arange(8)) % 8]
    assert np.array_equal(flip, np.conj(xi))
    assert np.max(np.abs(ifftn(xi).imag)) < 1e-14
    assert not np.array_equal(xi, m.noise_hat(f, 4))


# ------------------------------------------------------------- nonlinear ---
def test_single_cosine_cube():
    lat = Lattice(48, 4)
    m = om.Model(lat, 0.01)
    f = m.add_field("phi")
    m.add_term(f, [Mono(1.0)], [(f, 3)])
    A, k0 = 0.8, 5
    x = np.arange(48)
    m.set_real(f, np.broadcast_to(A * np.cos(2 * np.pi * k0 * x / 48), lat.shape))
    N3 = m.nonlinear_hat(0)
    want = np.zeros(lat.shape, dtype=complex)
    for kk, amp in ((k0, 0.75), (3 * k0, 0.25)):
        want[0, 0, kk] += amp * A ** 3 * lat.N / 2
        want[0, 0, -kk] += amp * A ** 3 * lat.N / 2
    assert np.max(np.abs(N3 - want)) < 1e-12 * lat.N


def _exact_convolution(spec_list, kept_out):
    """Non-periodic convolution of the factors' retained modes at output modes."""
    shape = spec_list[0].shape
    nz, ny, nx = shape

    def signed(i, n):
        return i - n if i >= (n + 1) // 2 else i
    modes = []
    for s in spec_list:
        lst = []
        for idx in zip(*np.nonzero(s)):
            kv = tuple(signed(i, n) for i, n in zip(idx, shape))
            lst.append((kv, s[idx]))
        modes.append(lst)
    out = {}
    for combo in itertools.product(*modes):
        ksum = tuple(sum(c[0][d] for c in combo) for d in range(3))
        val = np.prod([c[1] for c in combo])
        out[ksum] = out.get(ksum, 0) + val
    N = nx * ny * nz
    res = np.zeros(shape, dtype=complex)
    for idx in zip(*np.nonzero(kept_out)):
        kv = tuple(signed(i, n) for i, n in zip(idx, shape))
        res[idx] = out.get(kv, 0) / N ** (len(spec_list) - 1)
    return res


@pytest.mark.parametrize("shape", [SHAPE_RADIAL, SHAPE_PER_AXIS])
@pytest.mark.parametrize("order", [2, 3])
def test_order_rule_removes_aliasing(order, shape):
    lat = Lattice(12, 8)
    m = om.Model(lat, 0.01, dealias=DEALIAS_PAPER_ORDER, shape=shape)
    f = m.add_field("phi")
    m.add_term(f, [Mono(1.0)], [(f, order)])
    m.set_real(f, _rand_field(lat, 9))
    mask = lat.mask(2, order + 1, shape)
    spec = m.state[f] * mask
    got = m.nonlinear_hat(0)
    ref = _exact_convolution([spec] * order, mask)
    assert np.max(np.abs((got - ref)[mask])) < 1e-12 * np.max(np.abs(got))
    # without the mask the same comparison fails: aliasing is real
    if order == 3:
        small = Lattice(8, 4)
        m2 = om.Model(small, 0.01, dealias=om.DEALIAS_NONE)
        f2 = m2.add_field("phi")
        m2.add_term(f2, [Mono(1.0)], [(f2, order)])
        m2.set_real(f2, _rand_field(small, 9))
        full = np.ones(small.shape, bool)
        ref2 = _exact_convolution([m2.state[f2]] * order, full)
        assert np.max(np.abs(m2.nonlinear_hat(0) - ref2)) > 1e-3


def test_two_field_product_matches_convolution():
    lat = Lattice(8, 8)
    m = om.Model(lat, 0.01, dealias=DEALIAS_PAPER_ORDER)
    a = m.add_field("a")
    b = m.add_field("b")
    m.add_term(a, [Mono(1.0)], [(a, 1), (b, 2)])
    m.set_real(a, _rand_field(lat, 1))
    m.set_real(b, _rand_field(lat, 2))
    mask = lat.mask(1, 2)
    got = m.nonlinear_hat(0)
    ref = _exact_convolution([m.state[a] * mask, m.state[b] * mask, m.state[b] * mask], mask)
    assert np.max(np.abs((got - ref)[mask])) < 1e-12 * np.max(np.abs(got))


# --------------------------------------------------------------- Model B ---
def test_model_b_mass_is_bit_invariant():
    lat = Lattice(32, 32)
    m = om.model_b(lat, 0.01, D=0.01, seed=1)
    m.init_uniform(0, -0.1, 0.1)
    m0 = m.state[0][0, 0, 0]
    for _ in range(5):
        m.step(10)
        assert m.state[0][0, 0, 0] == m0


def test_initial_field_is_float32_uniform():
    lat = Lattice(64, 64)
    m = om.model_b(lat, 0.01)
    vals = m.init_uniform(0, -0.1, 0.1)
    assert np.all(vals.astype(np.float32).astype(np.float64) == vals)
    assert vals.min() >= -0.1 and vals.max() <= 0.1
    assert abs(vals.mean()) < 4 * 0.2 / np.sqrt(12 * vals.size)
    assert np.max(np.abs(m.real(0) - vals)) < 1e-15


@pytest.mark.parametrize("k,b", [(1.0, 1.0), (4.0, 2.0)])
def test_stationary_kink(k, b):
    a = -1.0
    nx, dx = 512, 0.25
    lat = Lattice(nx, 4, 1, dx=dx)
    L = nx * dx
    x = np.arange(nx) * dx
    w = np.sqrt(2 * k / (-a))
    amp = np.sqrt(-a / b)
    prof = -amp * np.tanh((x - L / 4) / w) * np.tanh((x - 3 * L / 4) / w)
    prof = np.broadcast_to(prof, lat.shape)
    m = om.model_b(lat, 0.01, a=a, b=b, k=k, D=0.0)
    m.set_real(0, prof)
    m.step(500)
    assert np.max(np.abs(m.real(0) - prof)) < 1e-3
    # a kink of the wrong width is not stationary
    bad = -amp * np.tanh((x - L / 4) / (1.3 * w)) * np.tanh((x - 3 * L / 4) / (1.3 * w))
    m2 = om.model_b(lat, 0.01, a=a, b=b, k=k, D=0.0)
    m2.set_real(0, np.broadcast_to(bad, lat.shape))
    m2.step(500)
    assert np.max(np.abs(m2.real(0) - bad)) > 1e-2


def test_free_energy_decreases():
    lat = Lattice(32, 32)
    m = om.model_b(lat, 0.01, D=0.0)
    m.set_real(0, _rand_field(lat, 8, 0.3))
    g = [ob.free_energy(lat, m.state[0], -1, 1, 1)]
    for _ in range(30):
        m.step(5)
        g.append(ob.free_energy(lat, m.state[0], -1, 1, 1))
    assert np.all(np.diff(g) < 0)


def test_translation_equivariance():
    lat = Lattice(16, 32)
    f0 = _rand_field(lat, 10, 0.5)
    m1 = om.model_b(lat, 0.01, D=0.0)
    m1.set_real(0, f0)
    m1.step(20)
    m2 = om.model_b(lat, 0.01, D=0.0)
    m2.set_real(0, np.roll(f0, (3, 5), axis=(1, 2)))
    m2.step(20)
    assert np.max(np.abs(np.roll(m1.real(0), (3, 5), axis=(1, 2)) - m2.real(0))) < 1e-13


def test_restart_is_exact_replay():
    lat = Lattice(16, 16)
    m = om.model_b(lat, 0.01, D=0.05, seed=3)
    m.init_uniform(0, -0.1, 0.1)
    r = m.copy()
    m.step(20)
    r.step(10)
    r2 = r.copy()
    r2.step(10)
    assert np.array_equal(m.state[0], r2.state[0])


def test_real_space_stays_real_with_noise():
    lat = Lattice(16, 8, 4)
    m = om.two_field_3d(lat, 0.005)
    m.init_uniform(0, -0.1, 0.1)
    m.init_uniform(1, -0.1, 0.1)
    m.step(5)
    for f in (0, 1):
        z = ifftn(m.state[f])
        assert np.max(np.abs(z.imag)) < 1e-14 * max(1, np.max(np.abs(z.real)))


def test_implicit_term_validation():
    lat = Lattice(8, 8)
    m = om.Model(lat, 0.1)
    a = m.add_field("a")
    b = m.add_field("b")
    with pytest.raises(ValueError):
        m.add_term(a, [Mono(1.0)], [(b, 1)], implicit=True)
    with pytest.raises(ValueError):
        m.add_term(a, [Mono(1.0)], [(a, 2)], implicit=True)
