"""Pins of the oracle adjoint (CPU only): FP64 central finite differences on
the four coefficients and on random directions of the initial field, and the
exactness of the terminal seed against differences of the loss."""

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import model as om
from oracle.spectral import Lattice, fftn


def _setup(n=16, nsteps=30, seed=4):
    lat = Lattice(n, n)
    m = om.model_b(lat, 0.01, seed=seed)
    mask = m._prepare()["masks"][0]
    x0 = m.init_uniform(0, -0.1, 0.1)
    phi0 = fftn(x0.astype(np.complex128))
    theta_star = (-1.0, 1.0, 1.0, 0.01)
    phiT, _ = adj.forward(lat, phi0, theta_star, 0.01, nsteps, seed, mask, store=False)
    from oracle import observables as ob
    S_star, _ = ob.shell_average(lat, ob.structure_factor(lat, phiT))
    return lat, mask, x0, phi0, S_star


def test_coefficient_gradients_match_central_differences():
    lat, mask, x0, phi0, S_star = _setup()
    theta = np.array([-0.9, 1.1, 0.9, 0.012])
    L, g, _ = adj.gradient(lat, phi0, theta, 0.01, 30, 4, mask, S_star)
    assert L > 0
    for i in range(4):
        h = 1e-4 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Lp = adj.loss(lat, adj.forward(lat, phi0, tp, 0.01, 30, 4, mask, False)[0], S_star)
        Lm = adj.loss(lat, adj.forward(lat, phi0, tm, 0.01, 30, 4, mask, False)[0], S_star)
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.max(np.abs(g))), (i, g[i], fd)


def test_initial_field_gradient_matches_directional_differences():
    lat, mask, x0, phi0, S_star = _setup()
    theta = np.array([-0.9, 1.1, 0.9, 0.012])
    _, _, gphi = adj.gradient(lat, phi0, theta, 0.01, 30, 4, mask, S_star)
    rng = np.random.default_rng(0)
    for _ in range(3):
        d = rng.standard_normal(lat.shape)
        h = 2e-6  # central differences converge as h^2 (next test)
        fp = fftn((x0 + h * d).astype(np.complex128))
        fm = fftn((x0 - h * d).astype(np.complex128))
        Lp = adj.loss(lat, adj.forward(lat, fp, theta, 0.01, 30, 4, mask, False)[0], S_star)
        Lm = adj.loss(lat, adj.forward(lat, fm, theta, 0.01, 30, 4, mask, False)[0], S_star)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(gphi * d))
        assert abs(an - fd) <= 1e-6 * abs(fd), (an, fd)


def test_differences_converge_to_the_adjoint_as_h_squared():
    lat, mask, x0, phi0, S_star = _setup()
    theta = np.array([-0.9, 1.1, 0.9, 0.012])
    _, _, gphi = adj.gradient(lat, phi0, theta, 0.01, 30, 4, mask, S_star)
    d = np.random.default_rng(1).standard_normal(lat.shape)
    an = float(np.sum(gphi * d))
    errs = []
    for h in (1e-3, 1e-4):
        Lp = adj.loss(lat, adj.forward(lat, fftn((x0 + h * d).astype(np.complex128)), theta, 0.01, 30, 4, mask,
                                       False)[0], S_star)
        Lm = adj.loss(lat, adj.forward(lat, fftn((x0 - h * d).astype(np.complex128)), theta, 0.01, 30, 4, mask,
                                       False)[0], S_star)
        errs.append(abs((Lp - Lm) / (2 * h) - an))
    assert 50 < errs[0] / errs[1] < 200  # a factor 100 for a tenfold smaller h


def test_gradient_vanishes_at_the_target():
    lat, mask, x0, phi0, S_star = _setup()
    L, g, gphi = adj.gradient(lat, phi0, (-1.0, 1.0, 1.0, 0.01), 0.01, 30, 4, mask, S_star)
    assert L == 0.0 and np.all(g == 0) and np.all(gphi == 0)


def test_terminal_seed_is_the_loss_derivative():
    lat, mask, x0, phi0, S_star = _setup(nsteps=5)
    rng = np.random.default_rng(3)
    phi = fftn(rng.standard_normal(lat.shape).astype(np.complex128))
    g = adj.loss_seed(lat, phi, S_star)
    d = fftn(rng.standard_normal(lat.shape).astype(np.complex128))
    h = 1e-6
    fd = (adj.loss(lat, phi + h * d, S_star) - adj.loss(lat, phi - h * d, S_star)) / (2 * h)
    assert abs(np.real(np.sum(np.conj(g) * d)) - fd) <= 1e-6 * abs(fd)


def test_stored_full_size_adjoint_matches_central_differences():
    """tests/golden/adjoint_256.json (written by make_adjoint_256.py from the
    oracle alone): at the adjoint workload's full size, 256^2 and 2000 steps,
    the adjoint gradient in (a, b, k, D) agrees with FP64 central differences
    of the loss (h = 1e-4 relative)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_256.json")
    with open(path) as f:
        doc = json.load(f)
    run = next(r for r in doc["runs"] if r["steps"] == doc["fd"]["steps"])
    g = np.array(run["grad"])
    fd = np.array(doc["fd"]["grad"])
    assert np.all(np.abs(g - fd) <= 1e-4 * np.abs(fd)), (g, fd)
    # coarsening moves the loss and the gradient up by orders of magnitude with the run length
    losses = [r["loss"] for r in doc["runs"]]
    assert all(b > 10 * a for a, b in zip(losses, losses[1:])), losses
