"""Benchmark of the SPECT OSEM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: OSEM at 128^3 voxels of 0.48 cm, 120 angles over 360 degrees,
128 x 128 bins, attenuation map (water cylinder 0.15/cm, bone rod 0.25/cm,
lung ellipsoids 0.04/cm), depth-dependent Gaussian collimator blur
sigma = 0.03 d + 0.1 cm, 20 hot spheres, Poisson data with 5e6 counts,
4 iterations x 8 subsets.  Synthetic, seeded data stand in for the paper's
clinical and Monte Carlo SPECT acquisitions (Section 3.1, Appendix A).

One step = one whole reconstruction with the data, the attenuation map and
the initial image already resident in HBM: the 8 subset sensitivities
H_m^T 1 and 32 subiterations (forward projection, ratio, back projection,
multiplicative update).  The timed region covers exactly K steps between
two device synchronisations.

value = voxel-angle projections per second, counting one forward plus one
adjoint application of a voxel-angle pair as one projection:
N^2 Nz A (I + 1/2) per reconstruction (the sensitivities are one adjoint
pass).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2309_01977_amd as S  # noqa: E402
from paper_2309_01977_amd import phantoms as P  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Bytes a projector must move per voxel-angle when every angle streams the
# object-space operands once: forward = activity + attenuation sample;
# adjoint = attenuation sample + object accumulator contribution.
BYTES_PER_VOXEL_ANGLE = 8.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def event_time_ms(fn, reps):
    """Mean duration of fn() on the current stream, from HIP events."""
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(w, f_true, mu):
    """The FP64 oracle on the host: one forward + adjoint pass over all angles."""
    from oracle import oracle as O
    O.build(force=False)
    og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
    f64, mu64 = f_true.astype(np.float64), mu.astype(np.float64)
    t0 = time.perf_counter()
    p = O.forward(og, f64, mu64)
    O.back(og, p, mu64)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.voxel_angles / dt, "unit": "voxel-angle projections/s (fwd+adj)",
            "cores": threads, "kind": "oracle",
            "sample": f"one FP64 forward + adjoint pass over all {w.n_angles} angles of the "
                      f"{w.n}^3 workload ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the reconstruction is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(2)

    w = P.C2
    torch.cuda.set_device(0)
    S.load_library()
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom(w)
    mu = torch.from_numpy(mu_np).cuda()
    ft = torch.from_numpy(f_true).cuda()
    gbar = plan.forward(ft, mu).cpu().numpy()
    _, noise = P.rngs(w.seed_index)
    g = torch.from_numpy(P.poisson_counts(gbar, w.total_counts, noise)).cuda()
    f = torch.empty(w.object_shape, device="cuda")
    log(f"workload {w.name}: data ready")

    def step():
        S.osem(plan, g, w.n_iters, w.n_subsets, mu, out=f)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(args.steps):
        step()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = float(per.mean())
    log(f"OSEM reconstruction: mean {ms:.3f} ms, wall {wall * 1e3 / args.steps:.3f} ms/step")

    pairs = w.voxel_angles * (w.n_iters + 0.5)
    value = pairs / (ms * 1e-3)

    # projector passes over all angles (forward, adjoint) for the roofline
    proj = torch.empty(w.proj_shape, device="cuda")
    back = torch.empty(w.object_shape, device="cuda")
    for _ in range(3):
        plan.forward(f, mu, out=proj)
        plan.back(proj, mu, out=back)
    t_fwd = event_time_ms(lambda: plan.forward(f, mu, out=proj), 20)
    t_adj = event_time_ms(lambda: plan.back(proj, mu, out=back), 20)
    bytes_fwd = BYTES_PER_VOXEL_ANGLE * w.voxel_angles
    achieved = bytes_fwd / (t_fwd * 1e-3) / 1e9
    log(f"forward pass {t_fwd:.3f} ms, adjoint pass {t_adj:.3f} ms")

    out = {
        "metric": "voxel-angle projections/s (fwd+adj) at 128^3x120; OSEM recon p50/p99 latency",
        "value": value,
        "unit": "voxel-angle projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nz": w.nz, "n_angles": w.n_angles,
                   "voxel_cm": w.voxel_cm, "attenuation": True,
                   "psf_sigma_cm": f"{w.psf_a}*d+{w.psf_b}", "iterations": w.n_iters,
                   "subsets": w.n_subsets, "counts": w.total_counts},
        "osem_latency_ms": {"p50": float(np.percentile(per, 50)),
                            "p99": float(np.percentile(per, 99))},
        "projector_pass_ms": {"fwd": t_fwd, "adj": t_adj,
                              "voxel_angles_per_s": w.voxel_angles / ((t_fwd + t_adj) * 1e-3)},
        "roofline": {"bound": "hbm", "kernel": "fwd_main (+fwd_reduce)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w, f_true, mu_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
