"""Write sq_stats_256.json: the FP64 oracle's shell-averaged structure factor
S_j(t) and domain length L(t) for 2D Model B coarsening on a 256x256 lattice,
averaged over 16 independent noise seeds.

Model B with a=-1, b=1, k=1, conserved noise D(q) = 0.01 q^2, dt = 0.01,
2/3 radial de-aliasing, initial field uniform[-0.1, 0.1] from each seed
(the coefficients of the 1024^2 workload, Sec. "Example"); snapshots at
t = 10, 20, 50, 100 (steps 1000, 2000, 5000, 10000).  S_j and L follow the definitions in
oracle/observables.py.  Calls nothing but the oracle.

Usage (about ten minutes on 8 cores): python tests/golden/make_sq_stats_256.py [--seeds A B] [--out PATH]
(--seeds 101 116 --out other.json draws a second, independent oracle ensemble:
the oracle-against-oracle spread that calibrates the pass bar.)
"""

import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N = 256
SEEDS = tuple(range(1, 17))
SNAP_STEPS = (1000, 2000, 5000, 10000)
COEF = dict(a=-1.0, b=1.0, k=1.0, D=0.01)
DT = 0.01


def run(seed):
    from oracle import model as om
    from oracle import observables as ob
    from oracle import spectral
    spectral.WORKERS = 1
    lat = spectral.Lattice(N, N)
    m = om.model_b(lat, DT, seed=seed, **COEF)
    m.init_uniform(0, -0.1, 0.1)
    out, done = [], 0
    for s in SNAP_STEPS:
        m.step(s - done)
        done = s
        phi_hat = m.state[0]
        sj, nj = ob.shell_average(lat, ob.structure_factor(lat, phi_hat))
        out.append((sj.tolist(), nj.tolist(), ob.domain_length(lat, phi_hat)))
    return out


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, nargs=2, default=(SEEDS[0], SEEDS[-1]))
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "sq_stats_256.json"))
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    seeds = tuple(range(args.seeds[0], args.seeds[1] + 1))
    with mp.Pool(args.procs) as pool:
        res = pool.map(run, seeds)
    snaps = []
    for i, s in enumerate(SNAP_STEPS):
        S = np.array([r[i][0] for r in res])
        L = np.array([r[i][2] for r in res])
        snaps.append({
            "step": s, "t": s * DT,
            "S_mean": S.mean(axis=0).tolist(),
            "S_se": (S.std(axis=0, ddof=1) / np.sqrt(len(seeds))).tolist(),
            "L_mean": float(L.mean()),
            "L_se": float(L.std(ddof=1) / np.sqrt(len(seeds))),
            "n_j": res[0][i][1],
        })
    doc = {"lattice": [N, N], "dt": DT, "coef": COEF, "seeds": list(seeds),
           "dealias": "2/3 radial", "init": "uniform[-0.1,0.1] from the seed", "snapshots": snaps}
    path = args.out
    with open(path, "w") as f:
        json.dump(doc, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
