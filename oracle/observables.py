"""Observables of a field (oracle; tests only).

The paper shows Model B coarsening only as snapshots (Fig. 1), so these are
the standard coarsening diagnostics of the field it integrates:

* mass M = sum_x phi(x) = Re phi_hat(0), conserved exactly when every term and
  the noise carry a q^2 factor (conserved dynamics, Sec. "Pseudo-spectral
  integration", remark on continuity equations);
* structure factor S(k) = (dV/N) |phi_hat(k)|^2, shell averages
  S_j = mean over modes with round(|kt|) = j for 1 <= j < min(N_i)/2, where
  |kt| is the Euclidean norm of the signed integer mode index;
* domain length L = 2 pi sum_j n_j S_j / sum_j n_j |q_j| S_j with n_j the
  shell population and |q_j| = 2 pi j / (N dx) (square lattices).
"""

import numpy as np


def mass(phi_hat):
    return float(phi_hat.reshape(-1)[0].real)


def structure_factor(lat, phi_hat):
    return (lat.dV / lat.N) * np.abs(phi_hat) ** 2


def shell_index(lat):
    kx, ky, kz = lat.k_int
    kk = np.sqrt((kx * kx + ky * ky + kz * kz).astype(np.float64))
    return np.broadcast_to(np.rint(kk).astype(np.int64), lat.shape)


def n_shells(lat):
    sizes = [n for n in (lat.nx, lat.ny, lat.nz) if n > 1]
    return min(sizes) // 2


def shell_average(lat, s):
    """Return (S_j, n_j) for j = 1 .. n_shells-1 (index 0 of the arrays is j=1)."""
    j = shell_index(lat).reshape(-1)
    nj = n_shells(lat)
    sel = (j >= 1) & (j < nj)
    sums = np.bincount(j[sel], weights=s.reshape(-1)[sel], minlength=nj)
    cnt = np.bincount(j[sel], minlength=nj)
    return sums[1:nj] / np.maximum(cnt[1:nj], 1), cnt[1:nj]


def domain_length(lat, phi_hat):
    s = structure_factor(lat, phi_hat)
    sj, nj = shell_average(lat, s)
    j = np.arange(1, n_shells(lat))
    qj = 2 * np.pi * j / (lat.nx * lat.dx)
    return float(2 * np.pi * np.sum(nj * sj) / np.sum(nj * qj * sj))


def free_energy(lat, phi_hat, a, b, k):
    """G = sum_x dV [a/2 phi^2 + b/4 phi^4 + k/2 |grad phi|^2] (Sec. "Example")."""
    phi = np.fft.ifftn(phi_hat).real
    grad2 = np.zeros(lat.shape)
    for i in range(3):
        gi = np.fft.ifftn(lat.iq[i] * phi_hat).real
        grad2 = grad2 + gi * gi
    return float(lat.dV * np.sum(0.5 * a * phi ** 2 + 0.25 * b * phi ** 4 + 0.5 * k * grad2))
