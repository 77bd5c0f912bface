"""The device reductions are exact and repeat bit for bit (through the C
interface).

Shell means of the structure factor (Sec. "Example": the shell average of
(dV/N)|phi_hat(k)|^2 over round(|k|) = j) are compared with the exactly
rounded sums (math.fsum) of the same FP64 terms formed from the device's own
FP32 spectrum, so the only differences left are the fixed-point rounding of
each term (2^-62 of the shell's largest) and the final conversion: 1e-13
relative, in every shell, also where a shell is 1e-30 of the largest (a
linearly damped run, whose high shells have decayed by many decades).
Repeated calls, twin lattices and the allocation-free call agree bit for
bit, and so do two adjoint sweeps of the same run.
"""

import math

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402


def _shell_terms(lat, field):
    """The FP64 terms w (dV/N)|phi_hat|^2 of each shell, from the downloaded
    half spectrum (a mode of an interior column counts for its conjugate
    partner too)."""
    sp = lat.spectrum(field)  # (z, y, kx) with kx = 0 .. Nx/2
    n = lat.n
    nx, ny = n[0], n[1]
    nz = n[2] if len(n) == 3 else 1
    sp = sp.reshape(nz, ny, nx // 2 + 1)
    N = nx * ny * nz
    ns = min(n) // 2
    x = sp.real.astype(np.float64)
    y = sp.imag.astype(np.float64)
    kx = np.arange(nx // 2 + 1)
    ky = np.where(np.arange(ny) < ny // 2, np.arange(ny), np.arange(ny) - ny)
    kz = np.where(np.arange(nz) < nz // 2, np.arange(nz), np.arange(nz) - nz) if nz > 1 else np.zeros(1, int)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kk = KX.astype(np.float64) ** 2 + KY ** 2 + KZ ** 2
    j = np.rint(np.sqrt(kk)).astype(int)
    w = np.where((KX == 0) | (KX == nx // 2), 1, 2)
    t = (x * x + y * y) * (1.0 / N)
    out = []
    for s in range(1, ns):
        sel = j == s
        out.append(np.concatenate([t[sel & (w == 1)], np.repeat(t[sel & (w == 2)], 2)]))
    return out


def _exact_shells(lat, field):
    """Shell means with each shell summed exactly (math.fsum)."""
    terms = _shell_terms(lat, field)
    cnt = np.array([t.size for t in terms], dtype=np.int64)
    S = np.array([math.fsum(t.tolist()) / t.size for t in terms])
    return S, cnt


def _damped(n, steps, seed=5):
    """Linear decay q^2 (a + k q^2) with a > 0, no cubic term and no noise:
    each mode shrinks by the factor 1/(1 + dt q^2 (a + k q^2)) a step, so after
    40 steps the highest shells are near 1e-25 of the lowest."""
    lat = pss.Lattice(n, dt=0.01, seed=seed)
    f, _ = pss.model_b(lat, a=1.0, b=0.0, k=1.0, D=0.0)
    lat.init_uniform(f, -0.2, 0.2)
    lat.step(steps)
    return lat, f


@pytest.mark.parametrize("n,steps", [((256, 256), 40), ((128, 64), 0), ((32, 32, 32), 40), ((64, 32, 16), 5)])
def test_shell_means_are_the_exact_sums_of_the_device_spectrum(n, steps):
    print(f"exact shells n={n} steps={steps}", flush=True)
    lat, f = _damped(n, steps)
    S, cnt = lat.structure_factor(f)
    Se, ce = _exact_shells(lat, f)
    assert np.array_equal(cnt, ce)
    assert np.all(Se > 0)
    rel = np.abs(S - Se) / Se
    assert np.max(rel) <= 1e-13, (np.argmax(rel), np.max(rel))
    if steps >= 40:
        # the range the sums cover: a fixed point shared by all shells would lose the small ones
        assert Se.min() <= 1e-20 * Se.max(), (Se.min(), Se.max())


@pytest.mark.parametrize("n", [(512, 512), (32, 64, 16), (1024,)])
def test_structure_factor_repeats_bitwise(n):
    print(f"repeat shells n={n}", flush=True)

    def run():
        lat = pss.Lattice(n, dt=0.01, seed=9)
        f, _ = pss.model_b(lat, D=0.05)
        lat.init_uniform(f, -0.1, 0.1)
        lat.step(25)
        return lat, f

    a, fa = run()
    b, fb = run()
    assert np.array_equal(a.spectrum(fa), b.spectrum(fb))
    S1, c1 = a.structure_factor(fa)
    S2, c2 = a.structure_factor(fa)
    S3, c3 = b.structure_factor(fb)
    S4, c4 = b.structure_factor_noalloc(fb)
    for S, c in ((S2, c2), (S3, c3), (S4, c4)):
        assert np.array_equal(S, S1)
        assert np.array_equal(c, c1)


def test_non_finite_shells():
    # one infinite site: its transform holds infinite and NaN modes
    lat = pss.Lattice((64, 64), dt=0.01, seed=2)
    f, _ = pss.model_b(lat)
    x = np.zeros((64, 64), dtype=np.float32)
    x[3, 7] = np.inf
    lat.upload(f, x)
    S, cnt = lat.structure_factor(f)
    terms = _shell_terms(lat, f)
    assert np.array_equal(cnt, [t.size for t in terms])
    # as a plain sum would give: NaN if a term is NaN, else +inf if one is
    for j, t in enumerate(terms):
        if np.isnan(t).any():
            assert np.isnan(S[j]), j
        elif np.isinf(t).any():
            assert S[j] == np.inf, j
    assert np.isnan(S).any()


def test_adjoint_sweeps_repeat_bitwise():
    n, nsteps = (128, 128), 20

    def run():
        lat = pss.Lattice(n, dt=0.01, seed=4)
        f, _ = pss.model_b(lat, a=-0.9, b=1.1, k=0.9, D=0.012)
        lat.init_uniform(f, -0.1, 0.1)
        return lat

    ref = pss.Lattice(n, dt=0.01, seed=4)
    f, _ = pss.model_b(ref)
    ref.init_uniform(f, -0.1, 0.1)
    ref.step(nsteps)
    S_star, _ = ref.structure_factor(f)
    L1, g1, p1 = run().adjoint_model_b(nsteps, S_star, ckpt_every=6)
    L2, g2, p2 = run().adjoint_model_b(nsteps, S_star, ckpt_every=6)
    assert L1 > 0
    assert L1 == L2
    assert np.array_equal(g1, g2)
    assert np.array_equal(p1, p2)
