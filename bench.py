#!/usr/bin/env python3
"""Benchmark: 2D Model B (Cahn-Hilliard with conserved noise), 1024x1024, FP32.

One "step" is one full time step of the pseudo-spectral integrator (forward
and inverse transforms, real-space cubic, Philox noise, semi-implicit update)
over the whole lattice.  Prints one JSON line with site-steps/s, the roofline
position of the dominant kernel (the update kernel, HBM-bound) and the FP64
CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Summary of the FETCH_SIZE / WRITE_SIZE counter runs of the update kernel on
# this workload; its traffic figure is reported only while the kernel sources
# and the launch geometry are the ones the counters were taken with.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_update_kernel_modelb_1024.txt")
KERNEL_SOURCES = ("pss_kernels.hip", "pss_device.h", "pss_kernels.h", "pss_plan.h")
N = (1024, 1024)
A, B, K, D, DT, SEED = -1.0, 1.0, 1.0, 0.01, 0.01, 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_02410_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(geometry):
    """HBM bytes per update-kernel launch from the committed counter summary,
    or None if it is missing or was taken on other kernel code or geometry."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.split(":", 1) for l in f.read().splitlines() if ":" in l)
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    if kv.get("geometry") != json.dumps(geometry, sort_keys=True):
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_baseline(steps, steps_1core=5):
    """The FP64 oracle on `steps` steps of the same workload (after one warm-up),
    on all host cores, and on `steps_1core` steps with one FFT worker."""
    from oracle import model as om
    from oracle import spectral
    cores = os.cpu_count() or 1
    sites = N[0] * N[1]

    def rate(workers, k):
        spectral.WORKERS = workers
        m = om.model_b(spectral.Lattice(*N), DT, a=A, b=B, k=K, D=D, seed=SEED)
        m.init_uniform(0, -0.1, 0.1)
        m.step(1)
        t0 = time.perf_counter()
        m.step(k)
        return sites * k / (time.perf_counter() - t0)
    value = rate(cores, steps)
    one = rate(1, steps_1core)
    return {"value": value, "unit": "site-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of the 1024x1024 Model B workload after 1 warm-up step "
                      f"(numpy FP64; the FFTs run on scipy.fft with {cores} workers, the elementwise "
                      f"steps are single-threaded numpy)",
            "single_core": {"value": one, "sample": f"{steps_1core} steps, scipy.fft with 1 worker"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--kernel-reps", type=int, default=2000)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=("modelb1024", "ensemble", "adjoint", "3d"), default="modelb1024",
                    help="modelb1024: one 1024^2 lattice (default); ensemble: 256x128^2 + 64x256^2 + "
                         "16x512^2 independent lattices in one batch, also timed one lattice per launch; "
                         "adjoint: gradient of the structure-factor loss through 2000 steps at 256^2; "
                         "3d: the two-field 256^3 system (Model B phi coupled to Model A psi)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="ensemble: keep the default launch geometry instead of pss_autotune's choice per size")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times with a plain device "
                         "copy (a known-size reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the lattice is not sharded.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2405_02410_amd as pss
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        return ensemble(args, pss)
    if args.workload == "adjoint":
        return adjoint(args, pss)
    if args.workload == "3d":
        return three_d(args, pss)

    lat = pss.Lattice(N, dt=DT, seed=SEED)
    f, _ = pss.model_b(lat, a=A, b=B, k=K, D=D)
    lat.init_uniform(f, -0.1, 0.1)
    log(f"bench: 2D Model B {N[0]}x{N[1]}, warmup {args.warmup}, steps {args.steps}")
    lat.step(args.warmup)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(args.steps)
    lat.sync()
    el = time.perf_counter() - t0
    sites = N[0] * N[1]
    value = sites * args.steps / el
    ms_per_step = 1e3 * el / args.steps
    log(f"bench: {ms_per_step * 1e3:.2f} us/step, {value:.4e} site-steps/s")
    mass = lat.mass(f)

    # roofline of the dominant kernel: HIP events around back-to-back launches
    kb = lat.kernel_bytes(pss.KERNEL_UPDATE)
    ms_k, kname = lat.time_kernel(pss.KERNEL_UPDATE, args.kernel_reps)
    xb = lat.kernel_bytes(pss.KERNEL_X)
    ms_x, xname = lat.time_kernel(pss.KERNEL_X, args.kernel_reps)
    achieved = kb / (ms_k * 1e-3) / 1e9
    log(f"bench: {kname} {ms_k * 1e3:.2f} us/launch, {kb / 1e6:.2f} MB -> {achieved:.0f} GB/s; "
        f"{xname} {ms_x * 1e3:.2f} us/launch, {xb / 1e6:.2f} MB -> {xb / (ms_x * 1e-3) / 1e9:.0f} GB/s")
    step_bytes = kb + xb
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(lat.geometry()),
                "kernel": kname, "bytes_per_launch": kb, "us_per_launch": round(ms_k * 1e3, 3),
                "step_bytes": step_bytes,
                "step_GBs": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1)}

    if args.copy_mib > 0:
        nbytes = args.copy_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_mib} MiB three times")
        del src, dst

    cpu = None
    if not args.no_cpu:
        log(f"bench: timing the oracle on {args.cpu_steps} steps")
        cpu = cpu_baseline(args.cpu_steps)

    out = {
        "metric": "site-steps/s", "value": value, "unit": "site-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D Model B 1024x1024 FP32, a=-1 b=1 k=1, conserved noise D=0.01 q^2, "
                               "dt=0.01, 2/3 radial de-aliasing, uniform[-0.1,0.1] initial field, seed 1",
                   "lattice": list(N), "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mass_after": mass,
    }
    print(json.dumps(out), flush=True)


ENSEMBLE = ((256, 128), (64, 256), (16, 512))  # (members, side)


def ensemble_cpu_baseline(steps):
    """The FP64 oracle on `steps` steps of one 512^2 member (after one warm-up)."""
    from oracle import model as om
    from oracle import spectral
    cores = os.cpu_count() or 1
    spectral.WORKERS = cores
    m = om.model_b(spectral.Lattice(512, 512), DT, a=A, b=B, k=K, D=D, seed=SEED)
    m.init_uniform(0, -0.1, 0.1)
    m.step(1)
    t0 = time.perf_counter()
    m.step(steps)
    dt = time.perf_counter() - t0
    return {"value": 512 * 512 * steps / dt, "unit": "site-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of one 512x512 member of the ensemble after 1 warm-up step "
                      f"(numpy FP64, scipy.fft with {cores} workers); members are independent, so the "
                      f"site-step rate carries over to the whole ensemble"}


def ensemble(args, pss):
    """Batched ensemble: every member in one batch (one update and one x launch
    per size class and step) against the same members stepped one lattice per
    launch sequence (pss_step on each, each on its own stream)."""
    def build():
        lats, seed = [], 1000
        for count, side in ENSEMBLE:
            for _ in range(count):
                lat = pss.Lattice((side, side), dt=DT, seed=seed)
                f, _ = pss.model_b(lat, a=A, b=B, k=K, D=D)
                if args.autotune:
                    lat.autotune(reps=20)  # measured once per size, then cached
                lat.init_uniform(f, -0.1, 0.1)
                lats.append(lat)
                seed += 1
        return lats
    lats = build()
    sites = sum(c * s * s for c, s in ENSEMBLE)
    batch = pss.Batch(lats)
    log(f"bench: ensemble of {len(lats)} lattices, {sites} sites, {batch.classes()[0]} classes")
    batch.step(args.warmup)
    batch.sync()
    t0 = time.perf_counter()
    batch.step(args.steps)
    batch.sync()
    el = time.perf_counter() - t0
    value = sites * args.steps / el
    ms_per_step = 1e3 * el / args.steps
    log(f"bench: batched {ms_per_step * 1e3:.1f} us/step, {value:.4e} site-steps/s")

    # one lattice per launch sequence: the same members, pss_step on each
    plain_steps = max(1, args.steps // 10)
    for lat in lats:
        lat.step(args.warmup)
    for lat in lats:
        lat.sync()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(plain_steps)
    for lat in lats:
        lat.sync()
    pel = time.perf_counter() - t0
    plain = sites * plain_steps / pel
    log(f"bench: plain {1e6 * pel / plain_steps:.1f} us/step, {plain:.4e} site-steps/s")

    # roofline of the kernel with the largest share of the batched step
    best = None
    for cls in range(batch.classes()[0]):
        for which in (pss.KERNEL_UPDATE, pss.KERNEL_X):
            ms, nbytes = batch.time_kernel(cls, which, args.kernel_reps)
            log(f"bench: class {cls} kernel {which}: {ms * 1e3:.2f} us/launch, {nbytes / 1e6:.2f} MB")
            if best is None or ms > best[0]:
                best = (ms, nbytes, cls, which)
    ms, nbytes, cls, which = best
    achieved = nbytes / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"{'update_kernel' if which == 0 else 'xrow_kernel'} (batched, size class {cls})",
                "bytes_per_launch": nbytes, "us_per_launch": round(ms * 1e3, 3)}
    cpu = None
    if not args.no_cpu:
        log("bench: timing the oracle on 10 steps of one 512^2 member")
        cpu = ensemble_cpu_baseline(10)
    out = {
        "metric": "site-steps/s", "value": value, "unit": "site-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ensemble of 2D Model B lattices, 256x128^2 + 64x256^2 + 16x512^2 FP32, "
                               "a=-1 b=1 k=1, D=0.01 q^2, dt=0.01, 2/3 radial de-aliasing, independent seeds, "
                               "one batch",
                   "members": len(lats), "sites": sites, "parallelism": "single GPU",
                   "geometry": "autotuned per size" if args.autotune else "default"},
        "plain": {"value": plain, "steps": plain_steps,
                  "form": "pss_step on each lattice in turn, each on its own stream"},
        "vs_plain": round(value / plain, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    batch.close()


def adjoint(args, pss):
    """Adjoint workload: dL/d(a, b, k, D) and dL/dphi_0 of the shell
    structure-factor loss after 2000 steps of 256^2 Model B, checkpoints every
    45 steps; the target spectrum comes from a forward run at (a, b, k, D) =
    (-1, 1, 1, 0.01), the gradient is taken at (-0.9, 1.1, 0.9, 0.012) with
    the same seed and initial field.  Compared with the plain forward run."""
    n, nsteps, ckpt = (256, 256), 2000, 45

    def make(theta):
        lat = pss.Lattice(n, dt=DT, seed=SEED)
        f, _ = pss.model_b(lat, a=theta[0], b=theta[1], k=theta[2], D=theta[3])
        lat.init_uniform(f, -0.1, 0.1)
        return lat
    ref = make((-1.0, 1.0, 1.0, 0.01))
    ref.step(nsteps)
    S_target, _ = ref.structure_factor(0)
    fwd = make((-0.9, 1.1, 0.9, 0.012))
    fwd.step(20)
    fwd.sync()
    t0 = time.perf_counter()
    fwd.step(nsteps)
    fwd.sync()
    t_fwd = time.perf_counter() - t0
    times = []
    for _ in range(3):
        lat = make((-0.9, 1.1, 0.9, 0.012))
        lat.sync()
        t0 = time.perf_counter()
        loss, grad, _ = lat.adjoint_model_b(nsteps, S_target, ckpt_every=ckpt)
        times.append(time.perf_counter() - t0)
    t_adj = min(times)
    sites = n[0] * n[1]
    log(f"bench: adjoint {t_adj * 1e3:.1f} ms for {nsteps} steps (forward alone {t_fwd * 1e3:.1f} ms); "
        f"loss {loss:.6g}, grad {grad}")
    out = {
        "metric": "site-steps/s", "value": sites * nsteps / t_adj, "unit": "site-steps/s", "n_gpus": 1,
        "steps": nsteps, "warmup": 20, "ms_per_step": 1e3 * t_adj / nsteps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "adjoint of 2D Model B 256x256 FP32 through 2000 steps, checkpoints every 45 "
                               "steps, structure-factor loss, gradients in (a, b, k, D) and phi_0",
                   "lattice": list(n), "parallelism": "single GPU"},
        "plain": {"value": sites * nsteps / t_fwd, "form": "the forward run alone (pss_step)"},
        "vs_plain": round(t_fwd / t_adj, 3),
        "loss": loss, "grad": list(grad),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def three_d(args, pss):
    """3D two-field system, 256^3 FP32: Model B phi (a, b, k = -1, 1, 1, conserved
    noise 0.005 q^2) coupled to non-conserved psi with
    d/dt psi = -(c psi + psi^3 - lap psi) - g phi psi + noise 0.005, and
    (g/2) phi psi^2 inside phi's chemical potential; c = -0.5, g = 0.3,
    dt = 0.005; launch geometry picked by pss_autotune."""
    from paper_2405_02410_amd import Mono
    n, dt, c, g, Dn = (256, 256, 256), 0.005, -0.5, 0.3, 0.005
    lat = pss.Lattice(n, dt=dt, seed=SEED)
    phi = lat.field("phi")
    psi = lat.field("psi")
    lat.term(phi, [Mono(-A, q2=1), Mono(-K, q2=2)], [(phi, 1)], implicit=True)
    lat.term(phi, [Mono(-B, q2=1)], [(phi, 3)])
    lat.term(phi, [Mono(-0.5 * g, q2=1)], [(phi, 1), (psi, 2)])
    lat.term(psi, [Mono(-c), Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    lat.term(psi, [Mono(-1.0)], [(psi, 3)])
    lat.term(psi, [Mono(-g)], [(phi, 1), (psi, 1)])
    lat.noise(phi, [Mono(Dn, q2=1)])
    lat.noise(psi, [Mono(Dn)])
    us_tuned = lat.autotune(reps=20)
    lat.init_uniform(phi, -0.1, 0.1)
    lat.init_uniform(psi, -0.1, 0.1)
    steps = min(args.steps, 2000)
    lat.step(args.warmup)
    lat.sync()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    el = time.perf_counter() - t0
    sites = n[0] * n[1] * n[2]
    names = ("update_kernel", "xrow_kernel", "ypass_kernel(inverse)", "ypass_kernel(forward)")
    best = None
    for w in range(lat.kernels_per_step()):
        ms, _ = lat.time_kernel(w, max(10, args.kernel_reps // 20))
        nb = lat.kernel_bytes(w)
        log(f"bench: {names[w]} {ms * 1e3:.1f} us/launch, {nb / 1e6:.1f} MB -> {nb / (ms * 1e-3) / 1e9:.0f} GB/s")
        if best is None or ms > best[0]:
            best = (ms, nb, names[w])
    ms, nb, kname = best
    achieved = nb / (ms * 1e-3) / 1e9
    log(f"bench: 3d {1e6 * el / steps:.1f} us/step, {sites * steps / el:.4e} site-steps/s")
    out = {
        "metric": "site-steps/s", "value": sites * steps / el, "unit": "site-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D two-field 256^3 FP32: Model B phi coupled to Model A psi, c=-0.5 g=0.3 "
                               "D=0.005, dt=0.005, 2/3 radial de-aliasing, uniform[-0.1,0.1] initial fields",
                   "lattice": list(n), "parallelism": "single GPU", "geometry": lat.geometry(),
                   "autotuned_kernel_us_per_step": round(us_tuned, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kname,
                     "bytes_per_launch": nb, "us_per_launch": round(ms * 1e3, 3)},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
