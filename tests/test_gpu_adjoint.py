"""GPU adjoint of 2D Model B (pss_adjoint_model_b) against the FP64 oracle
adjoint, which the CPU suite pins with central finite differences.

Tolerance: the GPU runs the trajectory and the reverse sweep in FP32 with
FP64 sums; gradients must agree with the oracle to 1e-3 relative (the stated
bar for the adjoint), the loss to 1e-4.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.spectral import Lattice as OLattice, fftn  # noqa: E402

THETA0 = (-0.9, 1.1, 0.9, 0.012)
THETA_STAR = (-1.0, 1.0, 1.0, 0.01)
DT = 0.01


def _oracle(n, nsteps, seed):
    lat = OLattice(n[0], n[1], 1)
    m = om.model_b(lat, DT, seed=seed)
    mask = m._prepare()["masks"][0]
    x0 = m.init_uniform(0, -0.1, 0.1)
    phi0 = fftn(x0.astype(np.complex128))
    phiT, _ = adj.forward(lat, phi0, THETA_STAR, DT, nsteps, seed, mask, store=False)
    S_star, _ = ob.shell_average(lat, ob.structure_factor(lat, phiT))
    L, g, gphi = adj.gradient(lat, phi0, np.array(THETA0), DT, nsteps, seed, mask, S_star)
    return S_star, L, g, gphi


def _gpu(n, seed, theta=THETA0):
    a, b, k, D = theta
    lat = pss.Lattice(n, dt=DT, seed=seed)
    f, _ = pss.model_b(lat, a=a, b=b, k=k, D=D)
    lat.init_uniform(f, -0.1, 0.1)
    return lat


def _check(L, g, gphi, Lo, go, gphio):
    assert abs(L - Lo) <= 1e-4 * abs(Lo), (L, Lo)
    scale = np.max(np.abs(go))
    for i in range(4):
        assert abs(g[i] - go[i]) <= 1e-3 * max(abs(go[i]), 1e-3 * scale), (i, g[i], go[i])
    assert np.max(np.abs(gphi - gphio)) <= 1e-3 * np.max(np.abs(gphio))


@pytest.mark.parametrize("n,nsteps,ckpt", [((64, 64), 30, 7), ((32, 64), 50, 45), ((64, 32), 12, 1)])
def test_adjoint_matches_the_oracle_adjoint(n, nsteps, ckpt):
    S_star, Lo, go, gphio = _oracle(n, nsteps, seed=4)
    lat = _gpu(n, seed=4)
    L, g, gphi = lat.adjoint_model_b(nsteps, S_star, ckpt_every=ckpt)
    _check(L, g, gphi, Lo, go, gphio)


def test_adjoint_256_full_size_against_the_oracle():
    n, nsteps = (256, 256), 200
    S_star, Lo, go, gphio = _oracle(n, nsteps, seed=2)
    lat = _gpu(n, seed=2)
    L, g, gphi = lat.adjoint_model_b(nsteps, S_star, ckpt_every=45)
    _check(L, g, gphi, Lo, go, gphio)


def test_checkpoint_spacing_changes_nothing_and_the_run_ends_forward():
    n, nsteps = (64, 64), 40
    S_star = _oracle(n, nsteps, seed=7)[0]
    out = []
    for ck in (1, 6, 40, 100):
        lat = _gpu(n, seed=7)
        out.append(lat.adjoint_model_b(nsteps, S_star, ckpt_every=ck))
        assert lat.step_index == nsteps
        twin = _gpu(n, seed=7)
        twin.step(nsteps)
        assert np.array_equal(lat.spectrum(0), twin.spectrum(0))
        lat.step(3)  # the lattice keeps stepping from the end of the run
        twin.step(3)
        assert np.array_equal(lat.spectrum(0), twin.spectrum(0))
    # the recomputed segments are the same steps and every sum is taken in a
    # fixed order (exact shell sums, per-block gradient slots): bitwise equal
    for L, g, gphi in out[1:]:
        assert L == out[0][0]
        assert np.array_equal(g, out[0][1])
        assert np.array_equal(gphi, out[0][2])


def test_gradient_vanishes_at_its_own_target():
    n, nsteps = (64, 64), 20
    ref = _gpu(n, seed=3, theta=THETA_STAR)
    ref.step(nsteps)
    S, _ = ref.structure_factor(0)
    L0, g0, gphi0 = _gpu(n, seed=3).adjoint_model_b(nsteps, S, ckpt_every=8)  # at theta0, for scale
    lat = _gpu(n, seed=3, theta=THETA_STAR)
    L, g, gphi = lat.adjoint_model_b(nsteps, S, ckpt_every=8)
    # the same trajectory and order-free shell sums: S_j equal bit for bit,
    # so the loss, its seed and every gradient are exactly zero
    assert L0 > 0 and np.max(np.abs(g0)) > 0 and np.max(np.abs(gphi0)) > 0
    assert L == 0.0
    assert np.all(g == 0.0)
    assert np.all(gphi == 0.0)


def test_noiseless_and_unsupported_models():
    n, nsteps = (32, 32), 10
    lat = pss.Lattice(n, dt=DT, seed=1)
    f, _ = pss.model_b(lat, D=0.0)
    lat.init_uniform(f)
    S = np.zeros(15)
    L, g, _ = lat.adjoint_model_b(nsteps, S, ckpt_every=4)
    assert L > 0 and g[3] == 0.0 and np.all(np.isfinite(g))
    bad = pss.Lattice(n, dt=DT)
    h = bad.field("h")
    bad.term(h, [pss.Mono(-1.0, q2=1)], [(h, 1)], implicit=True)
    bad.init_uniform(h)
    with pytest.raises(pss.PssError) as e:
        bad.adjoint_model_b(nsteps, S)
    assert e.value.name == "PSS_E_UNSUPPORTED"
    with pytest.raises(pss.PssError):
        lat.adjoint_model_b(nsteps, np.zeros(14))  # wrong shell count


def test_autograd_function_gives_the_adjoint_gradients():
    import torch
    from paper_2405_02410_amd.autograd import ModelBLoss
    n, nsteps, seed = (64, 64), 25, 5
    S_star, Lo, go, gphio = _oracle(n, nsteps, seed)
    lossf = ModelBLoss(n, DT, seed, nsteps, S_star, ckpt_every=10)
    x0 = om.model_b(OLattice(64, 64, 1), DT, seed=seed).init_uniform(0, -0.1, 0.1).reshape(64, 64)
    phi0 = torch.tensor(x0, dtype=torch.float32, device="cuda", requires_grad=True)
    theta = torch.tensor(THETA0, dtype=torch.float64, requires_grad=True)
    L = lossf(phi0, theta)
    (2.0 * L).backward()
    _check(L.item(), theta.grad.numpy() / 2, phi0.grad.cpu().numpy() / 2, Lo, go, gphio)
    # a second evaluation at other coefficients starts from the same step 0
    L2 = lossf(phi0.detach(), torch.tensor(THETA_STAR, dtype=torch.float64))
    assert L2.item() < 1e-3 * L.item()


def test_two_phase_tape_equals_the_one_call_and_guards_its_state():
    n, nsteps = (64, 64), 30
    S_star = _oracle(n, nsteps, seed=6)[0]
    L1, g1, gphi1 = _gpu(n, seed=6).adjoint_model_b(nsteps, S_star, ckpt_every=7)
    lat = _gpu(n, seed=6)
    L2, tape = lat.adjoint_forward(nsteps, S_star, ckpt_every=7)
    assert lat.step_index == nsteps
    gphi2 = np.empty(n[::-1], dtype=np.float32)
    g2 = tape.backward(gphi2)
    assert L2 == L1
    assert np.array_equal(g2, g1)
    assert np.array_equal(gphi2, gphi1)
    with pytest.raises(pss.PssError) as e:  # the sweep runs once
        tape.backward()
    assert e.value.name == "PSS_E_STATE"
    with pytest.raises(pss.PssError) as e:  # one tape per lattice at a time
        lat.adjoint_forward(nsteps, S_star)
    assert e.value.name == "PSS_E_STATE"
    with pytest.raises(pss.PssError) as e:
        lat.close()
    assert e.value.name == "PSS_E_STATE"
    tape.close()
    # a state change between the phases is refused
    L3, tape3 = lat.adjoint_forward(nsteps, S_star, ckpt_every=7)
    lat.step(1)
    with pytest.raises(pss.PssError) as e:
        tape3.backward()
    assert e.value.name == "PSS_E_STATE"
    tape3.close()


def test_autograd_forward_without_gradient_is_the_plain_run():
    import torch
    from paper_2405_02410_amd.autograd import ModelBLoss
    n, nsteps, seed = (64, 64), 25, 5
    S_star = _oracle(n, nsteps, seed)[0]
    lossf = ModelBLoss(n, DT, seed, nsteps, S_star, ckpt_every=10)
    x0 = om.model_b(OLattice(64, 64, 1), DT, seed=seed).init_uniform(0, -0.1, 0.1).reshape(64, 64)
    phi0 = torch.tensor(x0, dtype=torch.float32, device="cuda")
    theta = torch.tensor(THETA0, dtype=torch.float64)
    with torch.no_grad():
        L_plain = lossf(phi0, theta).item()
    assert lossf._tape is None
    L_rec = lossf(phi0.clone().requires_grad_(True), theta).item()
    assert lossf._tape is not None
    assert L_plain == L_rec
    # the gradient for phi0 comes back on the device
    p = phi0.clone().requires_grad_(True)
    lossf(p, theta).backward()
    assert p.grad.is_cuda and torch.isfinite(p.grad).all()


@pytest.mark.parametrize("nsteps", [500, 1000, 2000])
def test_adjoint_workload_256_against_the_stored_oracle(nsteps):
    """The adjoint workload at full size: 256^2, checkpoints every 45 steps,
    up to 2000 steps, against the FP64 oracle adjoint stored by
    tests/golden/make_adjoint_256.py (whose 2000-step gradient the CPU suite
    pins to central differences).  The GPU uses the oracle's target spectrum.

    The workload itself (2000 steps) must agree to 1e-3 per component
    (relative, or 1e-3 of the largest component for near-zero ones).  Shorter
    runs are a measurement of the FP32 limit: their loss is small (S stays
    close to S*), so the gradient 2 sum (S - S*) dS/dtheta magnifies the FP32
    separation of the trajectories (amplified in the linearly unstable band)
    relative to S - S*; at 500 steps the GPU gradient is held to 1e-2 of its
    largest component."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_256.json")
    with open(path) as f:
        doc = json.load(f)
    run = next(r for r in doc["runs"] if r["steps"] == nsteps)
    lat = _gpu(tuple(doc["lattice"]), seed=doc["seed"], theta=tuple(doc["theta0"]))
    L, g, gphi = lat.adjoint_model_b(nsteps, np.array(run["S_target"]), ckpt_every=45)
    go = np.array(run["grad"])
    scale = np.max(np.abs(go))
    rel = np.abs(g - go) / np.maximum(np.abs(go), 1e-3 * scale)
    print(f"n={nsteps}: loss {L:.8g} vs {run['loss']:.8g}; grad {g} vs {go}; relative {rel}", flush=True)
    sites = np.array(run["gphi0_sites"])
    dphi = np.max(np.abs(gphi[sites[:, 0], sites[:, 1]] - np.array(run["gphi0_at_sites"]))) / run["gphi0_absmax"]
    print(f"n={nsteps}: phi0 gradient at 64 sites, max error / max |grad| = {dphi:.3g}", flush=True)
    if nsteps >= 2000:
        assert abs(L - run["loss"]) <= 1e-3 * abs(run["loss"]), (L, run["loss"])
        assert np.all(rel <= 1e-3), rel
        assert dphi <= 1e-3
    else:
        assert abs(L - run["loss"]) <= 1e-2 * abs(run["loss"]), (L, run["loss"])
        assert np.all(np.abs(g - go) <= 1e-2 * scale), (g, go)
        assert dphi <= 1e-2
