"""Reverse-mode derivative of a Model B trajectory (oracle; tests only).

Forward (Sec. "Example" with conserved noise, stepped by eq:timeupdate):
    u_n        = Re F^-1[m . phi_n]                      (de-aliased factor)
    N_n        = F[u_n^3]
    eta_n      = sigma xi_n,  sigma = sqrt(2 D q^2 dt / dV)
    phi_{n+1}  = (phi_n + dt M N_n + eta_n) / A,   M = -b q^2,  A = 1 + dt q^2 (a + k q^2)
Loss on the final spectrum: L = sum_j (S_j - S*_j)^2 with the shell averages
S_j of the structure factor (dV/N)|phi_hat|^2 (j = 1 .. min(N_i)/2 - 1).

With the real inner product <x, y> = Re sum_k conj(x_k) y_k over all modes,
the adjoint g_n = dL/dphi_n obeys, per step taken backwards,
    r        = g_{n+1} / A
    wbar     = N Re F^-1[dt M r]
    ubar     = 3 u_n^2 wbar
    g_n      = r + m . F[ubar] / N
and the coefficients collect
    abar -= Re <r, dt q^2 phi_{n+1}>,   kbar -= Re <r, dt q^4 phi_{n+1}>,
    bbar += Re <r, -dt q^2 N_n>,        Dbar += Re <r, eta_n / (2 D)>.
The gradient with respect to the real initial field is N Re F^-1[g_0].
The noise xi_n is fixed by its Philox counter, so it is the same in every
evaluation (finite differences included).
"""

import numpy as np

from . import model as om
from . import observables as ob
from .spectral import fftn, ifftn


def _parts(m):
    """Model B pieces of an oracle model built by model.model_b."""
    c = m._prepare()
    lat = m.lat
    mask = c["masks"][0]
    return lat, mask, c


def coefficients_from(a, b, k, D, lat, dt):
    q2 = lat.q2
    A = 1.0 + dt * q2 * (a + k * q2)
    M = -b * q2
    sigma = np.sqrt(2.0 * D * q2 * dt / lat.dV) if D > 0 else np.zeros_like(q2)
    return A, M, sigma


def forward(lat, phi0_hat, theta, dt, nsteps, seed, mask, store=True):
    """Run Model B from phi0_hat with theta = (a, b, k, D); return the final
    spectrum and, if store, every intermediate spectrum."""
    a, b, k, D = theta
    A, M, sigma = coefficients_from(a, b, k, D, lat, dt)
    m = om.Model(lat, dt, seed=seed)
    f = m.add_field("phi")  # only used for its noise generator
    phi = phi0_hat.copy()
    hist = [phi.copy()] if store else None
    for n in range(nsteps):
        u = ifftn(phi * mask).real
        N = fftn((u ** 3).astype(np.complex128))
        eta = sigma * m.noise_hat(f, n) if D > 0 else 0.0
        phi = (phi + dt * M * N + eta) / A
        if store:
            hist.append(phi.copy())
    return phi, hist


def loss(lat, phi_hat, S_target):
    sj, _ = ob.shell_average(lat, ob.structure_factor(lat, phi_hat))
    return float(np.sum((sj - S_target) ** 2))


def loss_seed(lat, phi_hat, S_target):
    """dL/dphi_hat at the final step (the terminal adjoint)."""
    s = ob.structure_factor(lat, phi_hat)
    sj, nj = ob.shell_average(lat, s)
    j = ob.shell_index(lat)
    ns = ob.n_shells(lat)
    g = np.zeros(lat.shape, dtype=np.complex128)
    sel = (j >= 1) & (j < ns)
    coef = np.zeros(ns)
    coef[1:] = 2.0 * (sj - S_target) / np.maximum(nj, 1)
    g[sel] = coef[j[sel]] * (lat.dV / lat.N) * 2.0 * phi_hat[sel]
    return g


def gradient(lat, phi0_hat, theta, dt, nsteps, seed, mask, S_target):
    """Loss, d/d(a, b, k, D) and d/d(real phi_0) by the adjoint recursion."""
    a, b, k, D = theta
    A, M, sigma = coefficients_from(a, b, k, D, lat, dt)
    phiT, hist = forward(lat, phi0_hat, theta, dt, nsteps, seed, mask)
    L = loss(lat, phiT, S_target)
    g = loss_seed(lat, phiT, S_target)
    q2 = lat.q2
    m = om.Model(lat, dt, seed=seed)
    f = m.add_field("phi")
    ga = gb = gk = gD = 0.0
    for n in range(nsteps - 1, -1, -1):
        phin, phin1 = hist[n], hist[n + 1]
        u = ifftn(phin * mask).real
        N = fftn((u ** 3).astype(np.complex128))
        r = g / A
        ga -= float(np.real(np.sum(np.conj(r) * dt * q2 * phin1)))
        gk -= float(np.real(np.sum(np.conj(r) * dt * q2 * q2 * phin1)))
        gb += float(np.real(np.sum(np.conj(r) * (-dt * q2) * N)))
        if D > 0:
            eta = sigma * m.noise_hat(f, n)
            gD += float(np.real(np.sum(np.conj(r) * eta / (2.0 * D))))
        wbar = lat.N * ifftn(dt * M * r).real
        ubar = 3.0 * u * u * wbar
        g = r + mask * fftn(ubar.astype(np.complex128)) / lat.N
    gphi0 = lat.N * ifftn(g).real
    return L, np.array([ga, gb, gk, gD]), gphi0
