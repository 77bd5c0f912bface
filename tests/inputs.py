"""Seeded synthetic inputs shared by the oracle and GPU tests.

Holds none of the method's arithmetic: only random fields of given shapes and
amplitudes, and the model parameter sets of the workloads."""

import numpy as np


def random_field(shape, seed, amp=0.1, dtype=np.float32):
    """i.i.d. normal field (z, y, x) of standard deviation amp, rounded to dtype."""
    rng = np.random.default_rng(seed)
    return (amp * rng.standard_normal(shape)).astype(dtype)


def smooth_field(shape, seed, kmax=3, amp=0.3):
    """Sum of a few low Fourier modes (real), float32."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = np.zeros(shape)
    for _ in range(6):
        k = rng.integers(-kmax, kmax + 1, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        f += np.cos(2 * np.pi * (k[0] * x / nx + k[1] * y / ny + (k[2] * z / nz if nz > 1 else 0)) + ph)
    return (amp * f / 6).astype(np.float32)


# Model B coefficients of the 2D workloads (a, b, k, D, dt)
MODEL_B = dict(a=-1.0, b=1.0, k=1.0, D=0.01, dt=0.01)
