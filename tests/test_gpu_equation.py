"""Models written as equation strings (Sec. "Writing models") step on the GPU
bit for bit like the same models built with explicit C calls, and stay on the
FP64 oracle."""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402


def test_papers_model_b_example_string():
    # the example of Sec. "Example": a = -1, b = 1, k = 4, here with noise
    n, dt = (128, 128), 0.01
    s = pss.Lattice(n, dt=dt, seed=9)
    for name, v in (("a", -1.0), ("b", 1.0), ("k", 4.0), ("D", 0.01)):
        s.param(name, v)
    phi = s.field("phi")
    s.equation("dt phi + (a*q^2 + k*q^4)*phi = -b*q^2*phi^3")
    s.noise_expr(phi, "D*q^2")
    ref = pss.Lattice(n, dt=dt, seed=9)
    pss.model_b(ref, a=-1.0, b=1.0, k=4.0, D=0.01)
    for lat in (s, ref):
        lat.init_uniform(0, -0.1, 0.1)
        lat.step(80)
    assert np.array_equal(s.spectrum(0), ref.spectrum(0))
    m = om.model_b(OLattice(n[0], n[1], 1), dt, a=-1.0, b=1.0, k=4.0, D=0.01, seed=9)
    m.init_uniform(0, -0.1, 0.1)
    m.step(80)
    want = m.real(0)[0]
    assert np.max(np.abs(s.download(0) - want)) <= 1e-4 * max(1.0, np.max(np.abs(want)))


def test_kpz_strings_in_1d():
    n, dt = (256,), 0.01
    s = pss.Lattice(n, dt=dt, seed=3)
    s.param("sigma", 1.0)
    s.param("lambda", 0.5)
    phi = s.field("phi")
    s.field("dx_phi", dynamic=False)
    s.equation("dt phi + sigma*q^2*phi = 0")
    s.equation("dx_phi = iqx*phi")
    s.equation("dt phi = lambda*dx_phi^2")
    s.noise_expr(phi, "0.01")
    ref = pss.Lattice(n, dt=dt, seed=3)
    pss.kpz(ref, sigma=1.0, lam=0.5, D=0.01)
    for lat in (s, ref):
        lat.init_uniform(0, -0.5, 0.5)
        lat.step(60)
    assert np.array_equal(s.spectrum(0), ref.spectrum(0))
