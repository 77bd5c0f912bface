"""Pins of the oracle's observables (CPU only): a single Fourier mode has its
whole structure factor in one shell and a domain length of one wavelength;
the mass is the spatial sum."""

import numpy as np

from oracle import observables as ob
from oracle.spectral import Lattice, fftn


def test_single_mode_shell_and_length():
    lat = Lattice(64, 64, 1, dx=0.5, dy=0.5)
    x = np.arange(64) * 0.5
    k0 = 6
    f = np.broadcast_to(np.cos(2 * np.pi * k0 * x / 32.0), lat.shape)
    fh = fftn(f + 0j)
    sj, nj = ob.shell_average(lat, ob.structure_factor(lat, fh))
    assert np.argmax(sj * nj) + 1 == k0
    assert np.isclose(np.sum(sj * nj), np.sum(ob.structure_factor(lat, fh)))
    assert np.isclose(ob.domain_length(lat, fh), 32.0 / k0)


def test_mass_is_sum():
    lat = Lattice(8, 16)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(lat.shape)
    assert np.isclose(ob.mass(fftn(f + 0j)), f.sum())


def test_shell_populations():
    lat = Lattice(32, 32)
    j = ob.shell_index(lat)
    # shell 1 holds exactly the 4 nearest modes plus the 4 diagonal ones with |k|=sqrt2 (rounds to 1)
    assert np.sum(j == 1) == 8
    _, nj = ob.shell_average(lat, np.ones(lat.shape))
    assert nj.sum() == np.sum((j >= 1) & (j < 16))


def test_stored_coarsening_statistics_coarsen():
    """The stored 256^2 oracle ensemble (tests/golden/make_sq_stats_256.py)
    shows Model B coarsening: the domain length grows and the structure-factor
    peak moves to smaller shells between t = 10, 20, 50 and 100; the shell
    populations are those of the 256^2 lattice."""
    import json
    import os
    from oracle import observables as ob
    from oracle.spectral import Lattice
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sq_stats_256.json")
    with open(path) as f:
        snaps = json.load(f)["snapshots"]
    L = [s["L_mean"] for s in snaps]
    peaks = [int(np.argmax(s["S_mean"])) for s in snaps]
    assert all(b > a for a, b in zip(L, L[1:])), L
    assert all(b < a for a, b in zip(peaks, peaks[1:])), peaks
    _, nj = ob.shell_average(Lattice(256, 256), np.ones((256, 256)))
    for s in snaps:
        assert s["n_j"] == nj.tolist()
