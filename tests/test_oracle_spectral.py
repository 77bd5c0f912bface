"""Pins of the oracle's transforms, masks and operators (CPU only).

The transforms are pinned to a brute-force O(N^2) DFT, the masks to exact
rational arithmetic on the rule of Sec. "De-aliasing", and the operators to
analytic derivatives of trigonometric fields (Sec. "Reserved keywords":
q^2 is -lap, iq_x is d/dx, 1/q divides by |q|).
"""

import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle.spectral import (Lattice, Mono, fftn, ifftn, SHAPE_PER_AXIS,
                             SHAPE_RADIAL)


def naive_dft(a):
    """Brute-force sum_x a(x) exp(-2 pi i sum_i k_i x_i / N_i)."""
    out = np.zeros(a.shape, dtype=np.complex128)
    ranges = [range(n) for n in a.shape]
    for k in itertools.product(*ranges):
        s = 0j
        for x in itertools.product(*ranges):
            ph = sum(ki * xi / ni for ki, xi, ni in zip(k, x, a.shape))
            s += a[x] * np.exp(-2j * np.pi * ph)
        out[k] = s
    return out


@pytest.mark.parametrize("shape", [(4, 4), (8, 8), (6, 10), (4, 4, 4), (1, 8)])
def test_fft_matches_naive_dft(shape):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = naive_dft(a)
    got = fftn(a)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))) * a.size
    back = ifftn(got)
    assert np.max(np.abs(back - a)) < 1e-13


def test_parseval():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((16, 12))
    A = fftn(a)
    assert np.isclose(np.sum(a * a), np.sum(np.abs(A) ** 2) / a.size, rtol=1e-13)


def _frac_mask(lat, num, den, shape):
    f = Fraction(num, den)
    keep = np.zeros(lat.shape, dtype=bool)
    dims = [(i, n) for i, n in enumerate((lat.nx, lat.ny, lat.nz)) if n > 1]
    for idx in itertools.product(*[range(n) for n in lat.shape]):
        z, y, x = idx
        ks = {0: x, 1: y, 2: z}
        vals = []
        for i, n in dims:
            k = ks[i]
            if k > n // 2 or (n % 2 == 0 and k == n // 2):
                k = k - n
            vals.append(Fraction(k, n // 2))
        if shape == SHAPE_RADIAL:
            keep[idx] = sum(v * v for v in vals) < f * f
        else:
            keep[idx] = all(abs(v) < f for v in vals)
    return keep


@pytest.mark.parametrize("n", [(8, 8, 1), (12, 6, 1), (16, 16, 1), (8, 4, 6)])
@pytest.mark.parametrize("frac", [(2, 3), (1, 2), (2, 5)])
@pytest.mark.parametrize("shape", [SHAPE_RADIAL, SHAPE_PER_AXIS])
def test_mask_matches_exact_rational_rule(n, frac, shape):
    lat = Lattice(*n)
    got = lat.mask(*frac, shape)
    ref = _frac_mask(lat, *frac, shape)
    assert np.array_equal(got, ref)


def test_mask_one_dimensional_paper_rule():
    # Sec. "De-aliasing": for order n zero |q| > 2 pi/((n+1) dx); N=64, dx=1.
    lat = Lattice(64)
    for order in (2, 3):
        m = lat.mask(2, order + 1)[0, 0]
        q = np.abs(2 * np.pi * lat.kt[0] / 64)
        cut = 2 * np.pi / (order + 1)
        assert np.all(m[q > cut] == 0)
        assert np.all(m[q < cut] == 1)
    # n=3 puts the mode |kt| = 16 exactly on the cutoff: it is zeroed
    m3 = lat.mask(1, 2)[0, 0]
    assert m3[16] == 0 and m3[15] == 1


def _grid(lat):
    z, y, x = np.meshgrid(np.arange(lat.nz) * lat.dz, np.arange(lat.ny) * lat.dy,
                          np.arange(lat.nx) * lat.dx, indexing="ij")
    return x, y, z


def test_operators_are_derivatives():
    lat = Lattice(32, 16, 1, dx=0.5, dy=0.7)
    x, y, _ = _grid(lat)
    Lx, Ly = 32 * 0.5, 16 * 0.7
    ax, ay = 2 * np.pi * 3 / Lx, 2 * np.pi * 2 / Ly
    f = np.sin(ax * x) * np.cos(ay * y)
    F = fftn(f + 0j)

    def apply(monos):
        return ifftn(lat.operator(monos) * F).real

    # iq_x -> d/dx
    assert np.allclose(apply([Mono(1, iq=(1, 0, 0))]), ax * np.cos(ax * x) * np.cos(ay * y), atol=1e-12)
    # iq_y -> d/dy
    assert np.allclose(apply([Mono(1, iq=(0, 1, 0))]), -ay * np.sin(ax * x) * np.sin(ay * y), atol=1e-12)
    # q^2 -> -lap ; q^4 -> lap lap ; iq_x^2 -> d2/dx2
    assert np.allclose(apply([Mono(1, q2=1)]), (ax ** 2 + ay ** 2) * f, atol=1e-11)
    assert np.allclose(apply([Mono(1, q2=2)]), (ax ** 2 + ay ** 2) ** 2 * f, atol=1e-10)
    assert np.allclose(apply([Mono(1, iq=(2, 0, 0))]), -ax ** 2 * f, atol=1e-11)
    # 1/q on a single |q| shell divides by |q|
    assert np.allclose(apply([Mono(1, invq=1)]), f / np.hypot(ax, ay), atol=1e-12)
    # sums of monomials add
    two = apply([Mono(2.0, q2=1), Mono(-1.5)])
    assert np.allclose(two, 2 * (ax ** 2 + ay ** 2) * f - 1.5 * f, atol=1e-11)


def test_operator_special_modes():
    lat = Lattice(8, 8)
    inv = lat.operator([Mono(1, invq=1)])
    assert inv[0, 0, 0] == 0  # 1/|q| reads as 0 at q = 0
    iqx = lat.operator([Mono(1, iq=(1, 0, 0))])
    assert np.all(iqx[:, :, 4] == 0)  # odd derivative vanishes on the Nyquist plane
    q2 = lat.operator([Mono(1, q2=1)])
    assert np.isclose(q2[0, 0, 4].real, np.pi ** 2)
    assert np.isclose(q2[0, 4, 4].real, 2 * np.pi ** 2)


def test_linear_index_and_negative():
    lat = Lattice(4, 6, 2)
    z, y, x = 1, 2, 3
    assert lat.lin[z, y, x] == (z * 6 + y) * 4 + x
    assert lat.lin_neg[z, y, x] == ((2 - z) % 2 * 6 + (6 - y) % 6) * 4 + (4 - x) % 4
