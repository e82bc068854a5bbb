"""Benchmark of the SPECT OSEM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
                    [--recon-only] [--pair-only] [--workload osem|unrolled|bsrem|batched|serving]
                    [--serve-seconds S] [--serve-runs both|continuous|single]

Default workload: the 128^3 voxel, 120-angle acquisition (0.48 cm voxels,
128 x 128 bins, attenuation map with a water cylinder 0.15/cm, a bone rod
0.25/cm and lung ellipsoids 0.04/cm, depth-dependent Gaussian collimator blur
sigma = 0.03 d + 0.1 cm, 20 hot spheres, Poisson data of 5e6 counts).
Synthetic, seeded data stand in for the paper's clinical and Monte Carlo
SPECT acquisitions (Section 3.1, Appendix A).

value (the metric of record) = N^2 Nz A / (t_fwd + t_adj): the forward
projection and the back projection of all 120 angles with the attenuation
map and the blur (spect_fwd, spect_back), each the median of 50 calls timed
with HIP events after 5 warm-up calls, inputs resident in HBM.

One step = one whole OSEM reconstruction (4 iterations x 8 subsets: the 8
subset sensitivities H_m^T 1, then 32 subiterations of forward projection,
ratio, back projection and multiplicative update) with the data, the
attenuation map and the initial image resident in HBM; the timed region
covers exactly K steps between two device synchronisations; ms_per_step is
their mean and osem_latency_ms their p50/p99.  The steps cycle through five
Poisson draws of the data (spawned seeds), the last step using the first.

roofline: the dominant kernel of a reconstruction (by total time), its
algorithmic bytes per launch (8 B per voxel-angle in each direction, with
attenuation; 4 B without) over its average launch duration (HIP events on
its own launch stream), against the 8 TB/s HBM peak; roofline_alu gives
the same kernel's algorithmic FLOPs against the FP32 vector peak.

cpu_baseline: the FP64 oracle on the host cores, the same operator pair on a
bounded sample (one subset's angles) at the host's thread count, median of
3, with a single-thread leg, the 64^3 x 60 workload and one whole oracle
reconstruction beside it; the oracle also projects the phantom for the
data of the timed steps, and the last timed reconstruction is compared with
the oracle's reconstruction of the same data (accuracy).

Beside the default line: the 64^3 x 60 workload (OSEM p50/p99 over 100
reconstructions, fwd/adj medians), and compact runs of the batched,
unrolled (differentiable) and BSREM-RDP workloads (next_rows; --no-extras
skips them).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
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
PAIR_WARMUP, PAIR_REPS = 5, 50
DRAWS = 5


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
    return w.with_mu and 4 * w.n_angles * slabs * 16 * w.n * w.n <= TABLE_LIMIT


def recon_work(w, kernel, table):
    """(FP32 FLOP, algorithmic bytes) that `kernel` performs over one whole
    reconstruction (sensitivities + n_iters x n_subsets subiterations).

    Bytes: the operator's compulsory operand traffic, 8 B per voxel-angle in
    each direction with attenuation (forward: the activity sample and the
    attenuation sample; adjoint: the attenuation sample and the contribution
    to the object), 4 B without; the adjoint's bytes are split between its
    two kernels as the rotated-frame pass (attenuation) and the gather
    (object contribution).
    FLOP per voxel-angle: the separable depth-dependent blur costs 2 (2K+1)
    along each detector axis; a bilinear sample 7, the attenuation exponent
    5, a product 1; the gather 9 candidates x (weight 9 + 1 FMA)."""
    blur = float(np.mean([4 * (2 * k + 1) for k in blur_radii(w)]))
    va, it = float(w.voxel_angles), w.n_iters
    att_b = 4.0 if w.with_mu else 0.0
    if kernel == "fwd_main":
        flop = (8.0 if table or not w.with_mu else 20.0) + blur
        return it * va * flop, it * va * (4.0 + att_b)
    if kernel == "back_rot":
        sens = 13.0 + blur
        step = (1.0 + blur) if table or not w.with_mu else (13.0 + blur)
        return va * (sens + it * step), (it + 1) * va * att_b
    if kernel == "back_gather":
        return (it + 1) * va * 99.0, (it + 1) * va * 4.0
    return None, None


def per_call_ms(fn, warmup, reps):
    """Duration of each of `reps` back-to-back calls of fn (HIP events on the
    current stream, which the library launches on) after `warmup` calls."""
    for _ in range(warmup):
        fn()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    evs[0].record(st)
    for i in range(reps):
        fn()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    return np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(reps)])


def pair_metric(w, plan, f, mu):
    """Whole-angle forward and back projection: medians of PAIR_REPS calls
    after PAIR_WARMUP, and the voxel-angle rate of the pair."""
    proj = torch.empty(w.proj_shape, device="cuda")
    back = torch.empty(w.object_shape, device="cuda")
    plan.forward(f, mu, out=proj)
    tf = per_call_ms(lambda: plan.forward(f, mu, out=proj), PAIR_WARMUP, PAIR_REPS)
    tb = per_call_ms(lambda: plan.back(proj, mu, out=back), PAIR_WARMUP, PAIR_REPS)
    mf, mb = float(np.median(tf)), float(np.median(tb))
    return {"fwd_ms": mf, "adj_ms": mb,
            "fwd_p99_ms": float(np.percentile(tf, 99)), "adj_p99_ms": float(np.percentile(tb, 99)),
            "calls": PAIR_REPS, "warmup": PAIR_WARMUP,
            "voxel_angles_per_s": w.voxel_angles / ((mf + mb) * 1e-3),
            "fwd_voxel_angles_per_s": w.voxel_angles / (mf * 1e-3),
            "adj_voxel_angles_per_s": w.voxel_angles / (mb * 1e-3)}


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


def omp_threads():
    """Threads the oracle's OpenMP loops use: OMP_NUM_THREADS, else every
    CPU this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS")
    if v and v.isdigit():
        return int(v)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


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


# ----------------------------------------------------------- oracle legs ----

def oracle_pair_seconds(w, n_angles, reps, seed=0):
    """Seconds of the oracle's forward + back projection over the first
    n_angles angles of subset 0 of w (random inputs of the workload's shape:
    the oracle's time does not depend on the values), `reps` times."""
    O = _oracle()
    og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
    r = np.random.default_rng(seed)
    f = r.random(og.object_shape)
    mu = 0.15 * r.random(og.object_shape) if w.with_mu else None
    y = r.random(og.proj_shape)
    idx = list(range(0, w.n_angles, w.n_subsets))[:n_angles]
    out = []
    for _ in range(reps):
        t0 = time.perf_counter()
        O.forward(og, f, mu, idx)
        O.back(og, y, mu, idx)
        out.append(time.perf_counter() - t0)
    return out


def oracle_child_main(spec):
    """--oracle-sample NAME:ANGLES:REPS, run in a child process whose
    OMP_NUM_THREADS the parent set: prints the seconds of each repetition."""
    name, na, reps = spec.split(":")
    w = {"C1": P.C1, "C2": P.C2}[name]
    print(json.dumps({"seconds": oracle_pair_seconds(w, int(na), int(reps))}), flush=True)


def oracle_single_thread(name, n_angles, reps):
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", f"{name}:{n_angles}:{reps}"],
                       env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"single-thread oracle leg failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])["seconds"]


def leg(w, n_angles, secs):
    med = float(np.median(secs))
    va = w.n * w.n * w.nz * n_angles
    return {"angles": n_angles, "seconds": [round(x, 4) for x in secs], "median_s": med,
            "voxel_angles_per_s": va / med}


def cpu_baseline_legs(threads):
    """The oracle's operator pair on bounded samples: at the host's thread
    count (one subset of the 128^3 workload, the whole 64^3 workload) and on
    one thread (4 and 30 angles), each the median of 3."""
    log(f"oracle timing legs ({threads} threads, then 1 thread)")
    c2 = leg(P.C2, 15, oracle_pair_seconds(P.C2, 15, 3))
    c1 = leg(P.C1, 60, oracle_pair_seconds(P.C1, 60, 3))
    c2_1 = leg(P.C2, 4, oracle_single_thread("C2", 4, 3))
    c1_1 = leg(P.C1, 30, oracle_single_thread("C1", 30, 3))
    return {"value": c2["voxel_angles_per_s"], "unit": "voxel-angle projections/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(), "logical_cpus": os.cpu_count(),
            "sample": f"FP64 oracle forward + back projection of one subset (15 of 120 angles) of the "
                      f"128^3 workload with attenuation and blur, {threads} threads, median of 3: "
                      f"{c2['median_s']:.2f} s",
            "legs": {"osem_128cube_120ang_att": {"threads": threads, **c2},
                     "osem_128cube_120ang_att_1thread": {"threads": 1, **c2_1},
                     "osem_64cube_60ang": {"threads": threads, **c1},
                     "osem_64cube_60ang_1thread": {"threads": 1, **c1_1}}}


# ------------------------------------------------------ default workload ----

def small_workload(cpu):
    """The 64^3 x 60-angle workload (no attenuation, 2 it x 6 subsets): OSEM
    latency p50/p99 over 100 reconstructions, the operator pair, and (cpu)
    the last reconstruction against the oracle's."""
    w = P.C1
    plan = S.Plan.for_workload(w)
    f_true, _ = P.make_phantom(w)
    ft = torch.from_numpy(f_true).cuda()
    _, noise = P.rngs(w.seed_index)
    if cpu:
        O = _oracle()
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        gbar = O.forward(og, f_true.astype(np.float64))
    else:
        gbar = plan.forward(ft).cpu().numpy()
    g_np = P.poisson_counts(gbar, w.total_counts, noise)
    g = torch.from_numpy(g_np).cuda()
    f = torch.empty(w.object_shape, device="cuda")
    per = per_call_ms(lambda: S.osem(plan, g, w.n_iters, w.n_subsets, out=f), 5, 100)
    out = {"workload": w.name, "osem_latency_ms": {"p50": float(np.percentile(per, 50)),
                                                   "p99": float(np.percentile(per, 99)),
                                                   "reconstructions": 100},
           "voxel_angle_projections_per_s_osem": w.voxel_angles * (w.n_iters + 0.5) / (float(np.median(per)) * 1e-3),
           "projector_pair": pair_metric(w, plan, f, None)}
    if cpu:
        got = f.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        ref = O.osem(og, g_np.astype(np.float64), None, w.n_iters, w.n_subsets)
        out["oracle_osem_s"] = time.perf_counter() - t0
        out["rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return out


def bench_pair(args):
    """The metric of record alone: the whole-angle forward and back
    projection of the default workload's phantom with its attenuation map
    (no data, no reconstruction, no oracle), for profiler runs."""
    w = P.C2
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom(w)
    pair = pair_metric(w, plan, torch.from_numpy(f_true).cuda(), torch.from_numpy(mu_np).cuda())
    log(f"fwd {pair['fwd_ms']:.3f} ms, adj {pair['adj_ms']:.3f} ms (medians of {PAIR_REPS}): "
        f"{pair['voxel_angles_per_s']:.3e} voxel-angles/s")
    print(json.dumps({"metric": "voxel-angle projections/s (fwd+adj), pair-only run",
                      "value": pair["voxel_angles_per_s"], "projector_pair": pair}), flush=True)


def bench_osem(args):
    w = P.C2
    cpu = not args.no_cpu_baseline and not args.recon_only
    args.steps = 50 if args.steps is None else args.steps
    args.warmup = 3 if args.warmup is None else args.warmup
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom(w)
    mu = torch.from_numpy(mu_np).cuda()
    ft = torch.from_numpy(f_true).cuda()
    _, noise = P.rngs(w.seed_index)
    if cpu:
        O = _oracle()
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        t0 = time.perf_counter()
        gbar = O.forward(og, f_true.astype(np.float64), mu_np.astype(np.float64))
        t_orc_fwd = time.perf_counter() - t0
        source = "the FP64 oracle's projection of the phantom"
    else:
        gbar = plan.forward(ft, mu).cpu().numpy()
        source = "the library's projection of the phantom"
    draws = [P.poisson_counts(gbar, w.total_counts, noise) for _ in range(1 if args.recon_only else DRAWS)]
    gs = [torch.from_numpy(d).cuda() for d in draws]
    f = torch.empty(w.object_shape, device="cuda")
    log(f"workload {w.name}: data ready ({source}, {len(draws)} Poisson draws)")

    def step(k=0):
        S.osem(plan, gs[k % len(gs)], w.n_iters, w.n_subsets, mu, out=f)

    for i in range(args.warmup):
        step(i)
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(args.steps):
        step(args.steps - 1 - i)   # the last step reconstructs draw 0
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = float(per.mean())
    log(f"OSEM reconstruction: mean {ms:.3f} ms (events), {wall * 1e3 / args.steps:.3f} ms (wall)")
    if args.recon_only:
        print(json.dumps({"metric": "OSEM reconstructions (recon-only run)", "ms_per_step": ms,
                          "steps": args.steps, "warmup": args.warmup}), flush=True)
        return
    last = f.cpu().numpy().astype(np.float64)

    # the metric of record: the whole-angle operator pair
    pair = pair_metric(w, plan, ft, mu)
    log(f"fwd {pair['fwd_ms']:.3f} ms, adj {pair['adj_ms']:.3f} ms (medians of {PAIR_REPS}): "
        f"{pair['voxel_angles_per_s']:.3e} voxel-angles/s")
    with S.KernelTimer() as kt:
        proj = plan.forward(ft, mu)
        plan.back(proj, mu)
        torch.cuda.synchronize()
    pair["kernels"] = {k: {"launches": n, "avg_ms": t / n} for k, (n, t) in kt.stats().items()}

    # per-kernel durations of a reconstruction from HIP events on its stream
    kernels = kernel_stats(step, 3)
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    flop_r, bytes_r = recon_work(w, dom, uses_att_table(w))
    per_recon = kernels[dom]["launches"] / 3
    dur = kernels[dom]["avg_ms"] * 1e-3
    bytes_launch = bytes_r / per_recon
    gbs = bytes_launch / dur / 1e9
    tflops = flop_r / per_recon / dur / 1e12
    traffic = traffic_record(dom)
    log(f"dominant kernel {dom}: {kernels[dom]['avg_ms'] * 1e3:.1f} us/launch, "
        f"{gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.3f} of HBM), {tflops:.1f} TFLOP/s")
    small = small_workload(cpu)
    log(f"64^3 x 60 OSEM: p50 {small['osem_latency_ms']['p50']:.3f} ms")

    out = {
        "metric": "voxel-angle projections/s (fwd+adj) at 128^3x120; OSEM recon p50/p99 latency",
        "value": pair["voxel_angles_per_s"],
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
                   "subsets": w.n_subsets, "counts": w.total_counts, "data_source": source},
        "osem_latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                            "reconstructions": args.steps},
        "voxel_angle_projections_per_s_osem": w.voxel_angles * (w.n_iters + 0.5) / (ms * 1e-3),
        "projector_pair": pair,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": kernels[dom]["avg_ms"]},
        "roofline_alu": {"kernel": dom, "achieved": tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP32_VECTOR_PEAK_TFLOPS},
        "kernels": kernels,
        "small_workload": small,
    }
    if cpu:
        threads = omp_threads()
        log("oracle: the reconstruction of the last timed step's data")
        t0 = time.perf_counter()
        ref = O.osem(og, draws[0].astype(np.float64), mu_np.astype(np.float64), w.n_iters, w.n_subsets)
        t_orc_osem = time.perf_counter() - t0
        e = float(np.linalg.norm(last - ref) / np.linalg.norm(ref))
        log(f"last timed reconstruction vs the oracle's: rel L2 {e:.2e} (oracle {t_orc_osem:.1f} s)")
        out["accuracy"] = {"rel_l2_vs_oracle": e, "bar": 1e-4,
                           "rel_l2_vs_oracle_64cube": small.get("rel_l2_vs_oracle")}
        cb = cpu_baseline_legs(threads)
        cb["legs"]["osem_128cube_120ang_att_whole_reconstruction"] = {
            "threads": threads, "seconds": t_orc_osem,
            "voxel_angles_per_s": w.voxel_angles * (w.n_iters + 0.5) / t_orc_osem}
        cb["legs"]["forward_all_angles_for_the_data"] = {"threads": threads, "seconds": t_orc_fwd}
        out["cpu_baseline"] = cb
    if not args.no_extras:
        out["next_rows"] = {}
        for name, fn in (("batched", lambda: bench_batched(args, compact=True)),
                         ("unrolled", lambda: bench_unrolled(args, compact=True)),
                         ("bsrem", lambda: bench_bsrem(args, compact=True))):
            log(f"next row: {name}")
            out["next_rows"][name] = fn()
    print(json.dumps(out), flush=True)


def bench_unrolled(args, compact=False):
    """The differentiable workload: a batch of 8 torso phantoms at 128^3 with
    120 angles; one step = loss and gradient of 10 unrolled OSEM
    subiterations (8 subsets) from a uniform image, with checkpointing, loss =
    mean squared error to the phantoms.  The subset sensitivities are
    computed once before timing, together with each subset's
    attenuation-factor table (they depend on geometry and mu only); every
    projection in the timed region reads the tables."""
    w, B, K = P.C4, P.C4_BATCH, P.C4_STEPS
    steps = 2 if compact else (5 if args.steps is None else args.steps)
    warmup = 1 if compact else (1 if args.warmup is None else args.warmup)
    plan = S.Plan.for_workload(w)
    f_true, mu_np = P.make_phantom_batch(w, B, ss=2 if compact else 4)
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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(steps):
        step()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    ms = float(per.mean())
    log(f"unrolled loss + gradient, batch {B}: mean {ms:.2f} ms (events), {wall * 1e3 / steps:.2f} ms (wall)")
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
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
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
    if not args.no_cpu_baseline and not compact:
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
    return out


def bench_bsrem(args, compact=False):
    """BSREM-RDP (beta 0.3, gamma 2) on the 128^3, 120-angle data: one step =
    one whole reconstruction of 40 iterations x 8 subsets through
    bsrem_reconstruct (sensitivities and attenuation tables included)."""
    w = P.C6
    steps = 2 if compact else (3 if args.steps is None else args.steps)
    warmup = 1 if compact else (1 if args.warmup is None else args.warmup)
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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(st)
    for i in range(steps):
        step()
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    ms = float(per.mean())
    log(f"BSREM-RDP reconstruction: mean {ms:.2f} ms (events), {wall * 1e3 / steps:.2f} ms (wall)")
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
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
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
    if not args.no_cpu_baseline and not compact:
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
    return out


def bench_batched(args, compact=False):
    """32 uneven OSEM reconstructions (64^3 to 192x192x160, 60 to 128 angles,
    attenuation, 4 iterations x 8 subsets).  One step = all 32 reconstructed
    by one osem_batch_reconstruct call (autotuned schedule, graph-replayed
    iterations); the baseline runs the same 32 one at a time with
    osem_reconstruct.  Data, maps and initial images resident in HBM."""
    ws_ = P.c3_workloads()
    R = len(ws_)
    steps = 2 if compact else (3 if args.steps is None else args.steps)
    warmup = 1 if compact else (1 if args.warmup is None else args.warmup)
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

    per_single = timed(one_at_a_time, steps, warmup)
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

    per_batch = timed(batched, steps, warmup)
    per_sens = timed(lambda: batch.reconstruct(fs, mus, gs, 0), 2, 1)
    worst = max(float(((a - b).norm() / b.norm()).item()) for a, b in zip(fs, single))
    ms_b, ms_s = float(per_batch.mean()), float(per_single.mean())
    log(f"batched {ms_b:.1f} ms, one at a time {ms_s:.1f} ms, worst member difference {worst:.1e}")
    va = sum(w.voxel_angles * (w.n_iters + 0.5) for w in ws_)
    out = {
        "metric": "batched OSEM reconstructions/s (32 uneven geometries, 64^3..192x192x160, 60-128 angles)",
        "value": R / (ms_b * 1e-3),
        "unit": "reconstructions/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms_b,
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
    return out


def bench_serving(args):
    """A Poisson stream of 20 reconstruction requests per second for
    --serve-seconds seconds, each drawn from the 64^3 x 60 (no attenuation,
    2 x 6), 128^3 x 120 and 192 x 192 x 160 x 128 (attenuation, 4 x 8)
    classes with Poisson data (three noise draws per class), served by the
    continuous-batching server (up to 8 resident requests, 64 GiB pool) and,
    as the baseline, one request at a time through plain osem_reconstruct
    calls; then a burst of 60 requests at once (throughput), both ways."""
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
    # warm-up: one request of each class, both ways
    warm = S.Server(len(classes), 64 << 30)
    serving.replay(warm, classes, [(0.0, c) for c in range(len(classes))])
    warm.close()
    serving.replay_one_at_a_time(classes, [(0.0, c) for c in range(len(classes))])
    burst = [(0.0, int(c)) for c in rng.choice(len(classes), 60)]

    def run(name, trace_):
        t0 = time.perf_counter()
        if name == "one_at_a_time":
            served = serving.replay_one_at_a_time(classes, trace_, log_every_s=30.0)
            peak = 1
        else:
            server = S.Server(8, 64 << 30)
            served = serving.replay(server, classes, trace_, log_every_s=30.0)
            peak = server.stats()[2]
            server.close()
        wall = time.perf_counter() - t0
        st = serving.summary(served, wall)
        st["peak_resident"] = peak
        st["per_class_p50_ms"] = {classes[c].name: float(np.percentile(
            [s.latency * 1e3 for s in served if s.cls == c], 50)) for c in range(len(classes))
            if any(s.cls == c for s in served)}
        st["per_class_p99_ms"] = {classes[c].name: float(np.percentile(
            [s.latency * 1e3 for s in served if s.cls == c], 99)) for c in range(len(classes))
            if any(s.cls == c for s in served)}
        log(f"{name}: {st}")
        return st

    # --serve-runs picks one of the two ways (a 10-minute stream per way is
    # then one process each; the seeded trace and burst are the same)
    names = {"both": ("continuous_batching", "one_at_a_time"), "continuous": ("continuous_batching",),
             "single": ("one_at_a_time",)}[args.serve_runs]
    results = {}
    for name in names:
        results[name] = run(name, trace)
    for name in names:
        results["burst_" + name] = run(name, burst)
    cb = results.get("continuous_batching", results.get("one_at_a_time"))
    out = {
        "metric": "served OSEM reconstructions/s and p50/p99 latency (Poisson 20 req/s, 3 acquisition classes)",
        "value": cb["recon_per_s"],
        "unit": "reconstructions/s",
        "n_gpus": 1, "steps": len(trace), "warmup": len(classes), "ms_per_step": cb["latency_ms_mean"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving_poisson20", "classes": [c.name for c in classes],
                   "rate_per_s": P.C5_RATE, "seconds": args.serve_seconds, "max_resident": 8, "pool_gib": 64},
        "latency_ms_p50": cb["latency_ms_p50"], "latency_ms_p99": cb["latency_ms_p99"],
        "runs": results,
        "burst_throughput_ratio": (results["burst_continuous_batching"]["recon_per_s"] /
                                   results["burst_one_at_a_time"]["recon_per_s"]
                                   if len(names) == 2 else None),
    }
    if len(names) == 1:
        out["config"]["runs"] = names[0]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--recon-only", action="store_true")
    ap.add_argument("--pair-only", action="store_true",
                    help="time only the whole-angle projector pair of the default workload (for profiling)")
    ap.add_argument("--workload", choices=("osem", "unrolled", "bsrem", "batched", "serving"), default="osem")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-runs", choices=("both", "continuous", "single"), default="both")
    ap.add_argument("--oracle-sample", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_sample:
        oracle_child_main(args.oracle_sample)
        return
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
        print(json.dumps(bench_unrolled(args)), flush=True)
    elif args.workload == "bsrem":
        print(json.dumps(bench_bsrem(args)), flush=True)
    elif args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
    elif args.workload == "serving":
        bench_serving(args)
    elif args.pair_only:
        bench_pair(args)
    else:
        bench_osem(args)


if __name__ == "__main__":
    main()
