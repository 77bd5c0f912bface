"""Write adjoint_256.json: the FP64 oracle's structure-factor loss and its
gradients for 2D Model B on a 256x256 lattice, the adjoint workload.

Model B (Sec. "Example") with conserved noise, dt = 0.01, seed 1, initial field
uniform[-0.1, 0.1] from the seed, 2/3 radial de-aliasing.  The target spectrum
S*_j is the shell-averaged structure factor of a run at
theta* = (a, b, k, D) = (-1, 1, 1, 0.01); the loss
L = sum_j (S_j - S*_j)^2 and its gradient with respect to (a, b, k, D) and the
initial field are taken at theta0 = (-0.9, 1.1, 0.9, 0.012) with the same
seed and initial field, after n = 500, 1000 and 2000 steps
(oracle/adjoint.py).  For n = 2000 the four coefficient derivatives are also
taken by FP64 central differences of the oracle's loss (h = 1e-4 relative).
The gradient with respect to the initial field is stored at 64 fixed sites
(seeded) together with its largest magnitude.  Calls nothing but the oracle.

Usage (about fifteen minutes on 8 cores): python tests/golden/make_adjoint_256.py
"""

import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N = 256
DT = 0.01
SEED = 1
THETA_STAR = (-1.0, 1.0, 1.0, 0.01)
THETA0 = (-0.9, 1.1, 0.9, 0.012)
STEPS = (500, 1000, 2000)
FD_STEPS = 2000
H_REL = 1e-4
N_SITES = 64


def _setup():
    from oracle import model as om
    from oracle import spectral
    spectral.WORKERS = 1
    lat = spectral.Lattice(N, N)
    m = om.model_b(lat, DT, seed=SEED)
    mask = m._prepare()["masks"][0]
    x0 = m.init_uniform(0, -0.1, 0.1)
    phi0 = spectral.fftn(x0.astype(np.complex128))
    return lat, mask, phi0


def _target(nsteps):
    from oracle import adjoint as adj
    from oracle import observables as ob
    lat, mask, phi0 = _setup()
    phiT, _ = adj.forward(lat, phi0, THETA_STAR, DT, nsteps, SEED, mask, store=False)
    S, _ = ob.shell_average(lat, ob.structure_factor(lat, phiT))
    return S


def _gradient(nsteps):
    from oracle import adjoint as adj
    lat, mask, phi0 = _setup()
    S = _target(nsteps)
    L, g, gphi = adj.gradient(lat, phi0, np.array(THETA0), DT, nsteps, SEED, mask, S)
    rng = np.random.default_rng(256)
    sites = rng.integers(0, N, size=(N_SITES, 2))
    gp = gphi.reshape(N, N)
    return {"steps": nsteps, "S_target": S.tolist(), "loss": L, "grad": g.tolist(),
            "gphi0_sites": sites.tolist(), "gphi0_at_sites": [float(gp[y, x]) for y, x in sites],
            "gphi0_absmax": float(np.max(np.abs(gphi)))}


def _loss_at(args):
    from oracle import adjoint as adj
    i, sign = args
    lat, mask, phi0 = _setup()
    S = _target(FD_STEPS)
    th = np.array(THETA0, dtype=np.float64)
    h = H_REL * max(1.0, abs(th[i]))
    th[i] += sign * h
    phiT, _ = adj.forward(lat, phi0, tuple(th), DT, FD_STEPS, SEED, mask, store=False)
    return i, sign, h, adj.loss(lat, phiT, S)


def main():
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        fd_jobs = pool.map_async(_loss_at, [(i, s) for i in range(4) for s in (1, -1)])
        grads = pool.map(_gradient, STEPS)
        fd = fd_jobs.get()
    cd = [0.0] * 4
    for i in range(4):
        lp = next(v for j, s, h, v in fd if j == i and s == 1)
        lm = next(v for j, s, h, v in fd if j == i and s == -1)
        h = next(h for j, s, h, v in fd if j == i and s == 1)
        cd[i] = (lp - lm) / (2 * h)
    doc = {"lattice": [N, N], "dt": DT, "seed": SEED, "theta_star": THETA_STAR, "theta0": THETA0,
           "dealias": "2/3 radial", "init": "uniform[-0.1,0.1] from the seed",
           "runs": grads, "fd": {"steps": FD_STEPS, "h_rel": H_REL, "grad": cd}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_256.json")
    with open(path, "w") as f:
        json.dump(doc, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
