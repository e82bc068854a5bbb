"""Benchmark of the SPECT OSEM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--recon-only]
                    [--workload osem|unrolled|bsrem|batched|serving] [--serve-seconds S]

The default workload (osem) is the headline measurement below;
--workload unrolled measures the differentiable projector pair instead
(bench_unrolled), --workload bsrem BSREM with the relative difference prior
(bench_bsrem), --workload batched 32 uneven reconstructions at once against
the same reconstructions one at a time (bench_batched), --workload serving a
Poisson stream of reconstruction requests through the server (bench_serving).  --recon-only runs the data generation and the timed reconstructions only
(no per-kernel timing, context passes or CPU baseline); hardware-counter
runs use it so that every kernel they see after the data generation belongs
to a reconstruction.

Workload: OSEM at 128^3 voxels of 0.48 cm, 120 angles over 360 degrees,
128 x 128 bins, attenuation map (water cylinder 0.15/cm, bone rod 0.25/cm,
lung ellipsoids 0.04/cm), depth-dependent Gaussian collimator blur
sigma = 0.03 d + 0.1 cm, 20 hot spheres, Poisson data with 5e6 counts,
4 iterations x 8 subsets.  Synthetic, seeded data stand in for the paper's
clinical and Monte Carlo SPECT acquisitions (Section 3.1, Appendix A).

One step = one whole reconstruction with the data, the attenuation map and
the initial image already resident in HBM: the 8 subset sensitivities
H_m^T 1 and 32 subiterations (forward projection, ratio, back projection,
multiplicative update).  The timed region covers exactly K steps between two
device synchronisations.

value = voxel-angle projections per second, one forward plus one adjoint
application of a voxel-angle pair counted as one projection:
N^2 Nz A (I + 1/2) per reconstruction (the sensitivities are one adjoint
pass).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
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
from paper_2309_01977_amd.traffic import source_digest  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3
RDP_FLOP_PER_VOXEL = 26 * 13 + 5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_osem_128cube_120ang.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blur_radii(w):
    """Collimator blur radius K per depth (sigma = a d + b, K = ceil(4 sigma/dx))."""
    c = 0.5 * (w.n - 1)
    out = []
    for ip in range(w.n):
        d = max(0.0, 0.5 * w.n * w.voxel_cm - (ip - c) * w.voxel_cm)
        s = (w.psf_a * d + w.psf_b) / w.voxel_cm
        out.append(max(0, math.ceil(w.psf_nsigma * s - 1e-9)) if s > 0 else 0)
    return out


TABLE_LIMIT = 32 << 30   # the library keeps attenuation tables up to this total size


def uses_att_table(w):
    """Whether a whole reconstruction of w stores the attenuation factors of
    every subset (64 B per angle, 16-slice slab, depth and bin) and reads
    them back, as the library does while the tables fit in 32 GiB."""
    slabs = -(-w.nz // 16)
    return 4 * w.n_angles * slabs * 16 * w.n * w.n <= TABLE_LIMIT


def recon_work(w, kernel, table):
    """(FP32 FLOP, bytes) that `kernel` performs algorithmically over one
    whole reconstruction (sensitivities + n_iters x n_subsets subiterations).

    Per voxel-angle: the separable depth-dependent blur costs 2 (2K+1) FLOP
    along each detector axis.  Forward, sampling mu: two bilinear samples
    (activity, attenuation: 7 FLOP each), the attenuation exponent (5) and
    the product (1); bytes: the two samples.  Forward, reading the factor
    table: one bilinear sample (7) and the product (1); bytes: the sample and
    the factor.  Rotated-frame adjoint pass, sampling mu: one bilinear sample
    (7), the exponent (5) and the product (1); bytes: the mu sample and the
    rotated-frame value handed to the gather (+ the stored factor when it
    fills the table); reading the table: the product (1); bytes: factor and
    rotated-frame value.  Gather: 9 bilinear candidates x (weight 9 + 1 FMA);
    bytes: the rotated-frame value."""
    blur = float(np.mean([4 * (2 * k + 1) for k in blur_radii(w)]))
    va, it = float(w.voxel_angles), w.n_iters
    if kernel == "fwd_main":
        return (it * va * ((8.0 if table else 20.0) + blur), it * va * 8.0)
    if kernel == "back_rot":
        sens = (13.0 + blur, 12.0 if table else 8.0)
        step = (1.0 + blur, 8.0) if table else (13.0 + blur, 8.0)
        return (va * (sens[0] + it * step[0]), va * (sens[1] + it * step[1]))
    if kernel == "back_gather":
        return ((it + 1) * va * 99.0, (it + 1) * va * 4.0)
    return None, None


def event_ms(fn, reps):
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def traffic_record(kernel):
    """HBM bytes per reconstruction launch of `kernel`, measured with
    rocprofv3 counters, if they were taken on the current kernel sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("source_sha256") != source_digest():
            return None
        return rec["kernels"].get(kernel, {}).get("hbm_bytes_per_launch")
    except (OSError, ValueError, KeyError):
        return None


def _oracle():
    from oracle import oracle as O
    O.build(force=False)
    return O


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_workload():
    """The 64^3 x 60-angle workload (no attenuation, 2 it x 6 subsets): OSEM
    latency p50/p99 over 50 reconstructions and its projector passes."""
    w = P.C1
    plan = S.Plan.for_workload(w)
    f_true, _ = P.make_phantom(w)
    ft = torch.from_numpy(f_true).cuda()
    _, noise = P.rngs(w.seed_index)
    g = torch.from_numpy(P.poisson_counts(plan.forward(ft).cpu().numpy(), w.total_counts, noise)).cuda()
    f = torch.empty(w.object_shape, device="cuda")
    for _ in range(3):
        S.osem(plan, g, w.n_iters, w.n_subsets, out=f)
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(51)]
    torch.cuda.synchronize()
    evs[0].record(st)
    for i in range(50):
        S.osem(plan, g, w.n_iters, w.n_subsets, out=f)
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(50)])
    proj = torch.empty(w.proj_shape, device="cuda")
    back = torch.empty(w.object_shape, device="cuda")
    t_fwd = event_ms(lambda: plan.forward(f, out=proj), 20)
    t_adj = event_ms(lambda: plan.back(proj, out=back), 20)
    return {"workload": w.name, "osem_latency_ms": {"p50": float(np.percentile(per, 50)),
                                                    "p99": float(np.percentile(per, 99))},
            "voxel_angle_projections_per_s": w.voxel_angles * (w.n_iters + 0.5) / (float(per.mean()) * 1e-3),
            "projector_pass_ms": {"fwd": t_fwd, "adj": t_adj,
                                  "voxel_angles_per_s": w.voxel_angles / ((t_fwd + t_adj) * 1e-3)}}


def cpu_baseline(w, f_true, mu):
    """The FP64 oracle on the host: the same whole reconstruction, on data
    it projects itself (the same phantom and noise stream)."""
    O = _oracle()
    og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
    _, noise = P.rngs(w.seed_index)
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu.astype(np.float64)),
                         w.total_counts, noise)
    t0 = time.perf_counter()
    O.osem(og, g.astype(np.float64), mu.astype(np.float64), w.n_iters, w.n_subsets)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": w.voxel_angles * (w.n_iters + 0.5) / dt, "unit": "voxel-angle projections/s",
            "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"one whole FP64 OSEM reconstruction of the {w.n}^3 x {w.n_angles} workload "
                      f"({w.n_iters} it x {w.n_subsets} subsets, sensitivities included): {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--recon-only", action="store_true")
    ap.add_argument("--workload", choices=("osem", "unrolled", "bsrem", "batched", "serving"), default="osem")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(a reconstruction is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    S.load_library()
    # traffic calibration reference for counter runs: one plain 256 MiB device copy
    src = torch.zeros(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    if args.workload == "unrolled":
        bench_unrolled(args)
    elif args.workload == "bsrem":
        bench_bsrem(args)
    elif args.workload == "batched":
        bench_batched(args)
    elif args.workload == "serving":
        bench_serving(args)
    else:
        bench_osem(args)


def kernel_stats(run, reps):
    """Per-kernel launches and average duration from the library's own HIP
    events on the launch stream, over `reps` runs of `run`."""
    with S.KernelTimer() as kt:
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
    kstats = kt.stats()
    total = sum(v[1] for v in kstats.values())
    return {k: {"launches": n, "avg_ms": t / n, "share": t / total} for k, (n, t) in kstats.items()}


def bench_osem(args):
    w = P.C2
    args.steps = 20 if args.steps is None else args.steps
    args.warmup = 3 if args.warmup is None else args.warmup
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom(w)
    mu = torch.from_numpy(mu_np).cuda()
    ft = torch.from_numpy(f_true).cuda()
    gbar = plan.forward(ft, mu).cpu().numpy()
    _, noise = P.rngs(w.seed_index)
    g_np = P.poisson_counts(gbar, w.total_counts, noise)
    g = torch.from_numpy(g_np).cuda()
    f = torch.empty(w.object_shape, device="cuda")
    log(f"workload {w.name}: data ready")

    def step():
        S.osem(plan, g, w.n_iters, w.n_subsets, mu, out=f)

    for _ in range(args.warmup):
        step()
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
    log(f"OSEM reconstruction: mean {ms:.3f} ms (events), {wall * 1e3 / args.steps:.3f} ms (wall)")
    value = w.voxel_angles * (w.n_iters + 0.5) / (ms * 1e-3)
    if args.recon_only:
        print(json.dumps({"metric": "OSEM reconstructions (recon-only run)", "ms_per_step": ms,
                          "steps": args.steps, "warmup": args.warmup}), flush=True)
        return

    # per-kernel durations from HIP events the library records on its stream
    kernels = kernel_stats(step, 3)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    # per launch: one reconstruction's algorithmic work over its launches of
    # the kernel, divided by the average launch duration
    flop_r, bytes_r = recon_work(w, dom, uses_att_table(w))
    per_recon = kernels[dom]["launches"] / 3
    dur = kernels[dom]["avg_ms"] * 1e-3
    tflops = flop_r / per_recon / dur / 1e12
    gbs = bytes_r / per_recon / dur / 1e9
    traffic = traffic_record(dom)
    log(f"dominant kernel {dom}: {kernels[dom]['avg_ms'] * 1e3:.1f} us/launch, "
        f"{tflops:.1f} TFLOP/s, {gbs:.0f} GB/s algorithmic")

    # whole-angle projector passes (context)
    proj = torch.empty(w.proj_shape, device="cuda")
    back = torch.empty(w.object_shape, device="cuda")
    for _ in range(3):
        plan.forward(f, mu, out=proj)
        plan.back(proj, mu, out=back)
    t_fwd = event_ms(lambda: plan.forward(f, mu, out=proj), 10)
    t_adj = event_ms(lambda: plan.back(proj, mu, out=back), 10)
    small = small_workload()
    log(f"64^3 x 60 OSEM: p50 {small['osem_latency_ms']['p50']:.3f} ms")

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
        "roofline": {"bound": "alu", "kernel": dom, "achieved": tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic},
        "roofline_hbm": {"kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS},
        "kernels": kernels,
        "projector_pass_ms": {"fwd": t_fwd, "adj": t_adj,
                              "voxel_angles_per_s": w.voxel_angles / ((t_fwd + t_adj) * 1e-3)},
        "small_workload": small,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w, f_true, mu_np)
    print(json.dumps(out), flush=True)



def bench_unrolled(args):
    """The differentiable workload: a batch of 8 torso phantoms at 128^3 with
    120 angles; one step = loss and gradient of 10 unrolled OSEM
    subiterations (8 subsets) from a uniform image, with checkpointing, loss =
    mean squared error to the phantoms.  The subset sensitivities are
    computed once before timing, together with each subset's
    attenuation-factor table (they depend on geometry and mu only); every
    projection in the timed region reads the tables."""
    w, B, K = P.C4, P.C4_BATCH, P.C4_STEPS
    args.steps = 5 if args.steps is None else args.steps
    args.warmup = 1 if args.warmup is None else args.warmup
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom_batch(w, B)
    mu = torch.from_numpy(mu_np).cuda()
    tgt = torch.from_numpy(f_true).cuda()
    _, noise = P.rngs(w.seed_index)
    g = torch.stack([torch.from_numpy(P.poisson_counts(plan.forward(tgt[b], mu[b]).cpu().numpy(),
                                                       w.total_counts, noise)) for b in range(B)]).cuda()
    sens, tables = S.autograd.subset_sensitivities(plan, w.n_subsets, mu, tables=True)
    log(f"workload {w.name}: data ready")

    def step():
        f0 = torch.ones((B,) + w.object_shape, device="cuda", requires_grad=True)
        fk = S.unrolled_osem(plan, g, f0, K, w.n_subsets, mu, sens=sens, tables=tables)
        loss = ((fk - tgt) ** 2).mean(dim=(1, 2, 3)).sum()
        loss.backward()
        return f0.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(args.steps):
        step()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = float(per.mean())
    log(f"unrolled loss + gradient, batch {B}: mean {ms:.2f} ms (events), {wall * 1e3 / args.steps:.2f} ms (wall)")
    # projector passes per member: K forward subiterations (H, H^T) + K recomputed
    # in the backward pass + K backward (H^T of one adjoint, H of the other)
    passes = 6 * K
    sub_va = w.voxel_angles / w.n_subsets
    kernels = kernel_stats(step, 1)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    # per voxel-angle with the factors read from the tables (see recon_work)
    flop_va, bytes_va = {"fwd_main": (8.0, 8.0), "back_rot": (1.0, 8.0),
                         "back_gather": (99.0, 4.0)}.get(dom, (None, None))
    blur = float(np.mean([4 * (2 * k + 1) for k in blur_radii(w)]))
    if dom in ("fwd_main", "back_rot"):
        flop_va += blur
    dur = kernels[dom]["avg_ms"] * 1e-3
    tflops = flop_va * sub_va / dur / 1e12
    gbs = bytes_va * sub_va / dur / 1e9
    out = {
        "metric": "unrolled OSEM loss+gradient evaluations/s (batch 8, 128^3x120, 10 subiterations, checkpointed)",
        "value": B / (ms * 1e-3),
        "unit": "reconstruction gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "batch": B, "n": w.n, "nz": w.nz, "n_angles": w.n_angles,
                   "subsets": w.n_subsets, "unrolled_steps": K, "checkpointing": True,
                   "loss": "mean squared error to the phantom"},
        "voxel_angle_projections_per_s": B * passes * sub_va / (ms * 1e-3),
        "roofline": {"bound": "alu", "kernel": dom, "achieved": tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None},
        "roofline_hbm": {"kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS},
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle gradient of one member on the host")
        O = _oracle()
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        f0, m0 = f_true[0].astype(np.float64), mu_np[0].astype(np.float64)
        _, noise = P.rngs(w.seed_index)
        g0 = P.poisson_counts(O.forward(og, f0, m0), w.total_counts, noise).astype(np.float64)
        t0 = time.perf_counter()
        O.unrolled_osem_grad(og, g0, np.ones(w.object_shape), f0, K, w.n_subsets, m0)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / dt, "unit": "reconstruction gradients/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle",
                               "sample": f"one member's FP64 loss and gradient (sensitivities included): {dt:.1f} s"}
    print(json.dumps(out), flush=True)


def bench_bsrem(args):
    """BSREM-RDP (beta 0.3, gamma 2) on the 128^3, 120-angle data: one step =
    one whole reconstruction of 40 iterations x 8 subsets through
    bsrem_reconstruct (sensitivities and attenuation tables included)."""
    w = P.C6
    args.steps = 3 if args.steps is None else args.steps
    args.warmup = 1 if args.warmup is None else args.warmup
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom(w)
    mu = torch.from_numpy(mu_np).cuda()
    _, noise = P.rngs(w.seed_index)
    g = torch.from_numpy(P.poisson_counts(plan.forward(torch.from_numpy(f_true).cuda(), mu).cpu().numpy(),
                                          w.total_counts, noise)).cuda()
    f = torch.empty(w.object_shape, device="cuda")
    log(f"workload {w.name}: data ready")

    def step():
        f.fill_(1.0)
        plan.bsrem(g, w.n_iters, w.n_subsets, mu, f=f, beta=P.RDP_BETA, gamma=P.RDP_GAMMA)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(args.steps):
        step()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = float(per.mean())
    log(f"BSREM-RDP reconstruction: mean {ms:.2f} ms (events), {wall * 1e3 / args.steps:.2f} ms (wall)")
    kernels = kernel_stats(step, 1)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    flop_r, bytes_r = recon_work(w, dom, uses_att_table(w))
    per_recon = kernels[dom]["launches"]
    dur = kernels[dom]["avg_ms"] * 1e-3
    tflops = flop_r / per_recon / dur / 1e12
    gbs = bytes_r / per_recon / dur / 1e9
    # the prior stencil: reads the image and writes its gradient, 8 B per voxel
    rdp = kernels.get("rdp_grad")
    # the prior's gradient: per voxel 26 neighbour terms of 13 FLOP (an FMA
    # counted as 2, the reciprocal as 1) and 5 to combine the three distance
    # classes; 8 B of compulsory traffic (image read, gradient written)
    rdp_tflops = RDP_FLOP_PER_VOXEL * w.n * w.n * w.nz / (rdp["avg_ms"] * 1e-3) / 1e12 if rdp else None
    rdp_gbs = 8.0 * w.n * w.n * w.nz / (rdp["avg_ms"] * 1e-3) / 1e9 if rdp else None
    out = {
        "metric": "BSREM-RDP reconstruction latency at 128^3x120 (40 it x 8 subsets)",
        "value": ms,
        "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nz": w.nz, "n_angles": w.n_angles,
                   "iterations": w.n_iters, "subsets": w.n_subsets, "beta": P.RDP_BETA,
                   "gamma": P.RDP_GAMMA, "relaxation": "1/(1+k)"},
        "voxel_angle_projections_per_s": w.voxel_angles * (w.n_iters + 0.5) / (ms * 1e-3),
        "roofline": {"bound": "alu", "kernel": dom, "achieved": tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": None},
        "roofline_hbm": {"kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS},
        "prior_kernel": None if rdp is None else {
            "kernel": "rdp_grad", "avg_ms": rdp["avg_ms"], "bound": "alu", "achieved": rdp_tflops,
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": rdp_tflops / FP32_VECTOR_PEAK_TFLOPS,
            "hbm": {"achieved": rdp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rdp_gbs / HBM_PEAK_GBS}},
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("timing one FP64 oracle BSREM iteration on the host")
        O = _oracle()
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        _, noise = P.rngs(w.seed_index)
        g0 = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu_np.astype(np.float64)),
                              w.total_counts, noise).astype(np.float64)
        t0 = time.perf_counter()
        O.bsrem(og, g0, mu_np.astype(np.float64), 1, w.n_subsets, P.RDP_BETA, P.RDP_GAMMA)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dt * w.n_iters * 1e3, "unit": "ms",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle",
                               "sample": f"one FP64 iteration (8 subiterations, sensitivities included): {dt:.1f} s, "
                                         f"scaled to {w.n_iters} iterations"}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """32 uneven OSEM reconstructions (64^3 to 192x192x160, 60 to 128 angles,
    attenuation, 4 iterations x 8 subsets).  One step = all 32 reconstructed
    by one osem_batch_reconstruct call (autotuned schedule, graph-replayed
    iterations); the baseline runs the same 32 one at a time with
    osem_reconstruct.  Data, maps and initial images resident in HBM."""
    ws_ = P.c3_workloads()
    R = len(ws_)
    args.steps = 3 if args.steps is None else args.steps
    args.warmup = 1 if args.warmup is None else args.warmup
    plans = [S.Plan.for_workload(w) for w in ws_]
    mus, gs = [], []
    for i, (w, plan) in enumerate(zip(ws_, plans)):
        f_true, mu_np = P.make_member_phantom(w, i)
        mu = torch.from_numpy(mu_np).cuda()
        _, noise = P.member_rngs(i)
        gbar = plan.forward(torch.from_numpy(f_true).cuda(), mu).cpu().numpy()
        mus.append(mu)
        gs.append(torch.from_numpy(P.poisson_counts(gbar, w.total_counts, noise)).cuda())
    fs = [torch.empty(w.object_shape, device="cuda") for w in ws_]
    log(f"batched workload: {R} members ready")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record(st)
        for i in range(steps):
            fn()
            evs[i + 1].record(st)
        torch.cuda.synchronize()
        return np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])

    def one_at_a_time():
        for w, plan, f, mu, g in zip(ws_, plans, fs, mus, gs):
            S.osem(plan, g, w.n_iters, w.n_subsets, mu, out=f)

    per_single = timed(one_at_a_time, args.steps, args.warmup)
    single = [f.clone() for f in fs]
    for plan in plans:      # free the one-at-a-time workspaces
        plan._ws.clear()
    torch.cuda.empty_cache()
    batch = S.Batch(plans, ws_[0].n_subsets, True)
    for f in fs:
        f.fill_(1.0)
    sched, cand = batch.autotune(fs, mus, gs)
    log(f"autotuned schedule {sched}: ms per iteration {cand}")

    def batched():
        for f in fs:
            f.fill_(1.0)
        batch.reconstruct(fs, mus, gs, ws_[0].n_iters)

    per_batch = timed(batched, args.steps, args.warmup)
    per_sens = timed(lambda: batch.reconstruct(fs, mus, gs, 0), 2, 1)
    worst = max(float(((a - b).norm() / b.norm()).item()) for a, b in zip(fs, single))
    ms_b, ms_s = float(per_batch.mean()), float(per_single.mean())
    log(f"batched {ms_b:.1f} ms, one at a time {ms_s:.1f} ms, worst member difference {worst:.1e}")
    va = sum(w.voxel_angles * (w.n_iters + 0.5) for w in ws_)
    out = {
        "metric": "batched OSEM reconstructions/s (32 uneven geometries, 64^3..192x192x160, 60-128 angles)",
        "value": R / (ms_b * 1e-3),
        "unit": "reconstructions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "osem_batch32_uneven", "members": R, "iterations": ws_[0].n_iters,
                   "subsets": ws_[0].n_subsets, "attenuation": True, "schedule": sched,
                   "graph": True},
        "one_at_a_time": {"value": R / (ms_s * 1e-3), "unit": "reconstructions/s", "ms_per_step": ms_s},
        "speedup_vs_one_at_a_time": ms_s / ms_b,
        "voxel_angle_projections_per_s": va / (ms_b * 1e-3),
        "autotune_ms_per_iteration": cand,
        "batched_sensitivity_pass_ms": float(per_sens.mean()),
        "max_member_rel_l2_vs_one_at_a_time": worst,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """A Poisson stream of 20 reconstruction requests per second for
    --serve-seconds seconds, each drawn from the 64^3 x 60 (no attenuation,
    2 x 6), 128^3 x 120 and 192 x 192 x 160 x 128 (attenuation, 4 x 8)
    classes with Poisson data (three noise draws per class), served by the
    reconstruction server with 8 slots and a 64 GiB pool; the same trace
    served one request at a time (1 slot); and a burst of 60 requests at once
    (throughput) with 8 slots and with 1."""
    from paper_2309_01977_amd import serving
    works = [P.C1, P.C2, P.C5_LARGE]
    classes = []
    for w in works:
        plan = S.Plan.for_workload(w)
        f_true, mu_np = P.make_phantom(w, ss=2)
        mu = None if mu_np is None else torch.from_numpy(mu_np).cuda()
        gbar = plan.forward(torch.from_numpy(f_true).cuda(), mu).cpu().numpy()
        _, noise = P.rngs(w.seed_index)
        data = [torch.from_numpy(P.poisson_counts(gbar, w.total_counts, noise)).cuda() for _ in range(3)]
        classes.append(serving.RequestClass(w.name, plan, data, None if mu is None else [mu] * 3,
                                            w.n_iters, w.n_subsets))
    log("serving: request classes ready")
    rng = np.random.default_rng(np.random.SeedSequence(P.MASTER_SEED).spawn(5)[4].spawn(2)[1])
    trace = serving.poisson_trace(P.C5_RATE, args.serve_seconds, len(classes), rng)
    # warm-up: one request of each class
    warm = S.Server(len(classes), 64 << 30)
    serving.replay(warm, classes, [(0.0, c) for c in range(len(classes))])
    warm.close()
    results = {}
    for name, slots in (("server_8_slots", 8), ("one_at_a_time", 1)):
        server = S.Server(slots, 64 << 30)
        t0 = time.perf_counter()
        served = serving.replay(server, classes, trace)
        wall = time.perf_counter() - t0
        st = serving.summary(served, wall)
        st["peak_running"] = server.stats()[2]
        st["per_class_p99_ms"] = {classes[c].name: float(np.percentile(
            [s.latency * 1e3 for s in served if s.cls == c], 99)) for c in range(len(classes))
            if any(s.cls == c for s in served)}
        results[name] = st
        server.close()
        log(f"{name}: {st}")
    burst = [(0.0, int(c)) for c in rng.choice(len(classes), 60)]
    for name, slots in (("burst_8_slots", 8), ("burst_one_at_a_time", 1)):
        server = S.Server(slots, 64 << 30)
        t0 = time.perf_counter()
        served = serving.replay(server, classes, burst)
        wall = time.perf_counter() - t0
        results[name] = serving.summary(served, wall)
        results[name]["peak_running"] = server.stats()[2]
        server.close()
        log(f"{name}: {results[name]}")
    s8 = results["server_8_slots"]
    out = {
        "metric": "served OSEM reconstructions/s and p50/p99 latency (Poisson 20 req/s, 3 acquisition classes)",
        "value": s8["recon_per_s"],
        "unit": "reconstructions/s",
        "n_gpus": 1, "steps": len(trace), "warmup": len(classes), "ms_per_step": s8["latency_ms_mean"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_poisson20", "classes": [c.name for c in classes],
                   "rate_per_s": P.C5_RATE, "seconds": args.serve_seconds, "slots": 8, "pool_gib": 64},
        "latency_ms_p50": s8["latency_ms_p50"], "latency_ms_p99": s8["latency_ms_p99"],
        "runs": results,
        "burst_speedup": results["burst_one_at_a_time"]["latency_ms_max"] / results["burst_8_slots"]["latency_ms_max"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
