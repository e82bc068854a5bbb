"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar (from the workload statement): forward projections within 1e-5 relative
L2 per projection, back projections within 1e-5 relative L2 over the volume,
the FP32 adjoint identity within 1e-5, OSEM within 1e-4 relative L2 after the
full run.  Both sides read the same FP32 inputs; the oracle promotes them to
FP64.  Data for the OSEM cases (Poisson counts of the phantom's expected
projection) are made by the oracle.
"""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import phantoms as P

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-5
BACK_TOL = 1e-5
OSEM_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    S.load_library()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def both(n, nz, A, voxel=0.48, psf=(0.03, 0.1), angles=None, radius=None):
    og = O.Geometry(n, nz, A, voxel, psf[0], psf[1], 4.0, angles, radius)
    plan = S.Plan(n, nz, A, voxel, psf[0], psf[1], 4.0, angles, radius)
    return og, plan


def check_forward(og, plan, f, mu, idx=None, tol=FWD_TOL, label=""):
    ref = O.forward(og, f.astype(np.float64), None if mu is None else mu.astype(np.float64), idx)
    out = plan.forward(dev(f), None if mu is None else dev(mu), idx)
    got = host(out)
    rows = range(og.n_angles) if idx is None else idx
    worst = 0.0
    for n in rows:
        if np.linalg.norm(ref[n]) == 0:
            assert np.abs(got[n]).max() <= 1e-30, (label, n)
            continue
        e = rel_l2(got[n], ref[n])
        worst = max(worst, e)
        assert e <= tol, (label, n, e)
    say(f"  forward {label}: worst per-projection rel L2 {worst:.2e}")
    return got, ref


# ------------------------------------------------------- operator parity --

SMALL = [
    # n, nz, A, mu, psf, random angles
    (16, 8, 6, True, (0.03, 0.1), True),
    (37, 20, 5, True, (0.03, 0.1), True),     # ragged N, slab tail (Nz % 16 != 0)
    (24, 6, 4, True, (0.03, 0.1), True),      # Nz % 4 != 0: scalar loads
    (33, 17, 7, False, (0.03, 0.1), True),
    (20, 12, 8, True, (0.0, 0.0), False),     # no blur
    (1, 3, 2, False, (0.0, 0.0), False),      # one voxel column
    (48, 40, 3, True, (0.06, 0.2), True),     # wider blur class
    (64, 64, 10, True, (0.03, 0.1), False),
    (29, 1, 4, True, (0.03, 0.1), True),      # one slice: the axial blur keeps only its centre tap
    (16, 16, 3, True, (0.03, 0.1), True),     # exactly one full slab
]


@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}_nz{c[1]}_a{c[2]}_mu{int(c[3])}" for c in SMALL])
def test_forward_and_back_parity_small(case):
    n, nz, A, with_mu, psf, rand_ang = case
    say(f"case n={n} nz={nz} A={A} mu={with_mu} psf={psf}")
    r = np.random.default_rng(100 + n + nz + A)
    ang = list(r.uniform(0, 360, A)) if rand_ang else None
    og, plan = both(n, nz, A, psf=psf, angles=ang)
    f = P.random_object(og.object_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.2) if with_mu else None
    check_forward(og, plan, f, mu, label="all angles")
    idx = [A - 1, 0] if A > 1 else [0]
    check_forward(og, plan, f, mu, idx=idx, label="subset")
    y = P.random_object(og.proj_shape, r)
    ref = O.back(og, y.astype(np.float64), None if mu is None else mu.astype(np.float64))
    got = host(plan.back(dev(y), None if mu is None else dev(mu)))
    e = rel_l2(got, ref)
    say(f"  back rel L2 {e:.2e}")
    assert e <= BACK_TOL
    ref_s = O.back(og, y.astype(np.float64), None if mu is None else mu.astype(np.float64), idx)
    got_s = host(plan.back(dev(y), None if mu is None else dev(mu), idx))
    assert rel_l2(got_s, ref_s) <= BACK_TOL


def test_chunked_launch_matches_single_chunk():
    """A one-angle launch splits depth into chunks with attenuation offsets
    from the pre-pass; it must agree with the all-angle launch."""
    w = P.C2
    r = np.random.default_rng(5)
    plan = S.Plan.for_workload(w)
    f = dev(P.random_object(w.object_shape, r))
    mu = dev(P.random_mu(w.object_shape, r, 0.2))
    full = host(plan.forward(f, mu))
    for n in (0, 37, 119):
        one = host(plan.forward(f, mu, [n]))
        e = rel_l2(one[n], full[n])
        say(f"  angle {n}: chunked vs single-chunk rel L2 {e:.2e}")
        assert e <= 2e-6
    b_full = host(plan.back(dev(full), mu))
    b_one = sum(host(plan.back(dev(full), mu, [n])) for n in range(0, 120, 40))
    b_three = host(plan.back(dev(full), mu, list(range(0, 120, 40))))
    assert rel_l2(b_one, b_three) <= 2e-6
    assert np.isfinite(b_full).all()


@pytest.mark.parametrize("which", ["C1", "C2"])
def test_adjoint_identity_fp32(which):
    """<H x, y> = <x, H^T y> for the GPU pair at the full workload grids."""
    w = P.C1 if which == "C1" else P.C2
    r = np.random.default_rng(11)
    plan = S.Plan.for_workload(w)
    mu = dev(P.random_mu(w.object_shape, r, 0.2)) if w.with_mu else None
    for signed in (False, True):
        x = P.random_object(w.object_shape, r, signed)
        y = P.random_object(w.proj_shape, r, signed)
        hx = host(plan.forward(dev(x), mu))
        hty = host(plan.back(dev(y), mu))
        lhs = float(np.vdot(hx, y.astype(np.float64)))
        rhs = float(np.vdot(x.astype(np.float64), hty))
        scale = float(np.abs(hx).ravel() @ np.abs(y).ravel().astype(np.float64))
        e = abs(lhs - rhs) / scale
        say(f"  {which} signed={signed}: |<Hx,y> - <x,H^T y>| / scale = {e:.2e}")
        assert e <= 1e-5


def test_sensitivity_parity():
    w = P.C2
    r = np.random.default_rng(12)
    og, plan = both(w.n, w.nz, w.n_angles)
    mu = P.random_mu(w.object_shape, r, 0.2)
    idx = list(range(3, 120, 8))
    ref = O.back(og, np.ones(og.proj_shape), mu.astype(np.float64), idx)
    got = host(plan.sensitivity(dev(mu), idx))
    e = rel_l2(got, ref)
    say(f"  sensitivity rel L2 {e:.2e}")
    assert e <= BACK_TOL


@pytest.mark.parametrize("n,nz,A,with_mu", [(29, 19, 9, True), (16, 8, 6, False), (37, 20, 5, True), (1, 3, 2, True)],
                         ids=["odd_nz_mu", "no_mu", "ragged_n_mu", "one_column_mu"])
def test_sensitivity_parity_small(n, nz, A, with_mu):
    """H^T 1 of a random angle subset against the oracle: odd Nz takes the
    sensitivity pass's scalar loads, no map its attenuation-free form."""
    og, plan = both(n, nz, A, angles=list(np.random.default_rng(n).uniform(0, 360, A)))
    r = np.random.default_rng(13 + n)
    mu = P.random_mu(og.object_shape, r, 0.2) if with_mu else None
    idx = sorted(r.choice(A, size=max(1, A // 2), replace=False).tolist())
    ref = O.back(og, np.ones(og.proj_shape), None if mu is None else mu.astype(np.float64), idx)
    got = host(plan.sensitivity(None if mu is None else dev(mu), idx))
    e = rel_l2(got, ref)
    say(f"  n={n} nz={nz} A={A} mu={with_mu}: sensitivity rel L2 {e:.2e}")
    assert e <= BACK_TOL


def test_deterministic_results():
    """The gather-form back projection and the chunk reduction use a fixed
    summation order: repeated calls give identical bits."""
    w = P.C2
    r = np.random.default_rng(13)
    plan = S.Plan.for_workload(w)
    f = dev(P.random_object(w.object_shape, r))
    mu = dev(P.random_mu(w.object_shape, r, 0.2))
    idx = list(range(1, 120, 8))
    a = host(plan.forward(f, mu, idx))
    b = host(plan.forward(f, mu, idx))
    assert np.array_equal(a, b)
    y = dev(a)
    c = host(plan.back(y, mu, idx))
    d = host(plan.back(y, mu, idx))
    assert np.array_equal(c, d)


def test_empty_and_accumulating_calls():
    og, plan = both(16, 8, 4)
    r = np.random.default_rng(14)
    f = dev(P.random_object(og.object_shape, r))
    out = torch.full(og.proj_shape, 7.0, device="cuda")
    plan.forward(f, None, [], out=out)
    assert torch.all(out == 7.0)
    y = dev(P.random_object(og.proj_shape, r))
    b = torch.full(og.object_shape, 3.0, device="cuda")
    plan.back(y, None, [], out=b)
    assert torch.all(b == 0.0)
    base = plan.back(y, None, [0, 1]).clone()
    acc = base.clone()
    plan.back(y, None, [2, 3], out=acc, accumulate=True)
    full = plan.back(y, None)
    assert rel_l2(host(acc), host(full)) <= 1e-6


# --------------------------------------------------------- workload data --

_DATA = {}


def workload_data(w):
    if w.name not in _DATA:
        say(f"  building {w.name} phantom and oracle data")
        f_true, mu = P.make_phantom(w)
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        gbar = O.forward(og, f_true.astype(np.float64), None if mu is None else mu.astype(np.float64))
        _, noise = P.rngs(w.seed_index)
        g = P.poisson_counts(gbar, w.total_counts, noise)
        _DATA[w.name] = (og, f_true, mu, g)
    return _DATA[w.name]


@pytest.mark.parametrize("which", ["C1", "C2"])
def test_workload_forward_parity(which):
    w = P.C1 if which == "C1" else P.C2
    og, f_true, mu, _ = workload_data(w)
    plan = S.Plan.for_workload(w)
    check_forward(og, plan, f_true, mu, label=f"{which} all angles")
    check_forward(og, plan, f_true, mu, idx=list(range(0, w.n_angles, w.n_subsets)),
                  label=f"{which} subset 0")


def test_osem_step_conserves_counts_on_gpu():
    """P10 on the GPU: sum(sens_m f') = sum of g over the subset where Hf > 0."""
    w = P.C1
    og, f_true, mu, g = workload_data(w)
    plan = S.Plan.for_workload(w)
    M = w.n_subsets
    sens = S.sensitivities(plan, M, None)
    f = torch.ones(w.object_shape, device="cuda")
    gd = dev(g)
    for m in range(M):
        plan.osem_subset_step(f, gd, sens[m], m, M)
        idx = list(range(m, w.n_angles, M))
        lhs = float((sens[m].double() * f.double()).sum())
        rhs = float(g[idx].astype(np.float64).sum())
        assert abs(lhs - rhs) / rhs <= 1e-5, (m, lhs, rhs)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["C1", "C2"])
def test_osem_full_run_parity(which):
    """The whole reconstruction (sensitivities + I x M subiterations) against
    the FP64 oracle's OSEM on the same data: relative L2 <= 1e-4."""
    w = P.C1 if which == "C1" else P.C2
    og, f_true, mu, g = workload_data(w)
    plan = S.Plan.for_workload(w)
    got = host(S.osem(plan, dev(g), w.n_iters, w.n_subsets, None if mu is None else dev(mu)))
    say(f"  {which}: GPU OSEM done; running the oracle OSEM")
    ref = O.osem(og, g.astype(np.float64), None if mu is None else mu.astype(np.float64),
                 w.n_iters, w.n_subsets)
    e = rel_l2(got, ref)
    say(f"  {which}: OSEM rel L2 {e:.2e}")
    assert e <= OSEM_TOL


def test_noncircular_orbit_parity():
    """Irregular angles (negative, beyond 360 degrees, exact right angles) with
    a detector radius per angle (an elliptical orbit: every angle has its own
    blur radii and depth-chunk boundaries), with attenuation: the forward and
    back projections, the attenuation-table calls and a whole OSEM run against
    the oracle."""
    n, nz, A = 48, 24, 10
    ang = [-30.0, 0.0, 45.0, 90.0, 137.5, 180.0, 211.0, 270.0, 333.3, 400.0]
    rad = [12.0 + 8.0 * abs(np.cos(np.radians(t))) for t in ang]
    og, plan = both(n, nz, A, angles=ang, radius=rad)
    r = np.random.default_rng(77)
    f = P.random_object(og.object_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.15)
    mu64 = mu.astype(np.float64)
    check_forward(og, plan, f, mu, label="all angles")
    check_forward(og, plan, f, mu, idx=[9, 3, 4], label="subset")
    y = P.random_object(og.proj_shape, r)
    e_b = rel_l2(host(plan.back(dev(y), dev(mu))), O.back(og, y.astype(np.float64), mu64))
    idx = [1, 4, 7]
    sens_t, table = plan.sensitivity_table(dev(mu), idx)
    e_s = rel_l2(host(sens_t), O.back(og, np.ones(og.proj_shape), mu64, idx))
    fp = host(plan.forward_table(dev(f), table, idx))
    ref_f = O.forward(og, f.astype(np.float64), mu64, idx)
    worst = max(rel_l2(fp[i], ref_f[i]) for i in idx)
    e_bt = rel_l2(host(plan.back_table(dev(y), table, idx)), O.back(og, y.astype(np.float64), mu64, idx))
    say(f"  back {e_b:.2e}; table calls: sens {e_s:.2e}, forward worst {worst:.2e}, back {e_bt:.2e}")
    assert e_b <= BACK_TOL and e_s <= BACK_TOL and worst <= FWD_TOL and e_bt <= BACK_TOL
    g = P.poisson_counts(O.forward(og, f.astype(np.float64), mu64), 2e5, r)
    got = host(S.osem(plan, dev(g), 2, 5, dev(mu)))
    ref = O.osem(og, g.astype(np.float64), mu64, 2, 5)
    e = rel_l2(got, ref)
    say(f"  OSEM 2 x 5 rel L2 {e:.2e}")
    assert e <= OSEM_TOL


def test_osem_subset_extremes():
    """One angle per subset (n_subsets = n_angles: every launch lists a
    single angle), a single subset (plain MLEM), and zero iterations (only
    the sensitivities: the image stays as given, bitwise), against the
    oracle."""
    n, nz, A = 32, 20, 6
    og, plan = both(n, nz, A, angles=list(np.random.default_rng(8).uniform(0, 360, A)))
    r = np.random.default_rng(63)
    f_true = P.random_object(og.object_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.12)
    mu64 = mu.astype(np.float64)
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu64), 1e5, r)
    for I, M in ((2, A), (3, 1)):
        got = host(S.osem(plan, dev(g), I, M, dev(mu)))
        ref = O.osem(og, g.astype(np.float64), mu64, I, M)
        e = rel_l2(got, ref)
        say(f"  {I} it x {M} subsets: rel L2 {e:.2e}")
        assert e <= OSEM_TOL
    f0 = (0.5 + P.random_object(og.object_shape, r)).astype(np.float32)
    np.testing.assert_array_equal(host(S.osem(plan, dev(g), 0, 3, dev(mu), f0=dev(f0))), f0.astype(np.float64))


def test_one_plan_on_two_streams():
    """Projector calls with one plan issued on two streams at once (each
    stream gets its own scratch) give the results of the same calls one
    after another, bitwise."""
    og, plan = both(48, 32, 12)
    r = np.random.default_rng(62)
    fs = [dev(P.random_object(og.object_shape, r)) for _ in range(2)]
    mu = dev(P.random_mu(og.object_shape, r, 0.15))
    idx = [1, 5, 9]
    ref = [host(plan.forward(f, mu, idx)) for f in fs]
    ref_b = [host(plan.back(dev(x), mu, idx)) for x in ref]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = [[], []]
    for _ in range(4):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                p = plan.forward(fs[k], mu, idx)
                outs[k].append((p, plan.back(p, mu, idx)))
    torch.cuda.synchronize()
    for k in range(2):
        for p, b in outs[k]:
            np.testing.assert_array_equal(host(p), ref[k])
            np.testing.assert_array_equal(host(b), ref_b[k])


def test_repeated_angles_in_a_list():
    """An angle listed twice: the forward writes its row once more with the
    same values, the back projection and the sensitivity count it once per
    occurrence; against the oracle."""
    og, plan = both(24, 20, 8)
    r = np.random.default_rng(61)
    f = P.random_object(og.object_shape, r)
    y = P.random_object(og.proj_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.15)
    mu64 = mu.astype(np.float64)
    idx = [3, 6, 3, 3]
    got = host(plan.forward(dev(f), dev(mu), idx))
    ref = O.forward(og, f.astype(np.float64), mu64, idx)
    assert max(rel_l2(got[n], ref[n]) for n in (3, 6)) <= FWD_TOL
    assert not np.delete(got, [3, 6], axis=0).any()
    e_b = rel_l2(host(plan.back(dev(y), dev(mu), idx)), O.back(og, y.astype(np.float64), mu64, idx))
    e_s = rel_l2(host(plan.sensitivity(dev(mu), idx)), O.back(og, np.ones(og.proj_shape), mu64, idx))
    say(f"  repeated angles: back {e_b:.2e}, sensitivity {e_s:.2e}")
    assert e_b <= BACK_TOL and e_s <= BACK_TOL


def test_largest_grid_and_blur_radius():
    """At the limits the plan accepts: N = 256 (512-thread workgroups) and a
    blur radius of 32 pixels at the far depths (the widest blur class, whose
    rotated-frame pass needs more than 64 KB of LDS), with a slab tail
    (Nz = 20): projections, back projection, sensitivity and the table calls
    against the oracle."""
    n, nz, A = 256, 20, 3
    og, plan = both(n, nz, A, angles=[0.0, 33.0, 250.0])
    assert len(O.psf_taps(og, 0)) - 1 == 32
    r = np.random.default_rng(31)
    f = P.random_object(og.object_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.05)
    mu64 = mu.astype(np.float64)
    check_forward(og, plan, f, mu, label="n=256, K=32")
    y = P.random_object(og.proj_shape, r)
    e_b = rel_l2(host(plan.back(dev(y), dev(mu))), O.back(og, y.astype(np.float64), mu64))
    idx = [0, 2]
    sens_t, table = plan.sensitivity_table(dev(mu), idx)
    e_s = rel_l2(host(sens_t), O.back(og, np.ones(og.proj_shape), mu64, idx))
    fp = host(plan.forward_table(dev(f), table, idx))
    ref_f = O.forward(og, f.astype(np.float64), mu64, idx)
    worst = max(rel_l2(fp[i], ref_f[i]) for i in idx)
    e_bt = rel_l2(host(plan.back_table(dev(y), table, idx)), O.back(og, y.astype(np.float64), mu64, idx))
    say(f"  back {e_b:.2e}; table calls: sens {e_s:.2e}, forward worst {worst:.2e}, back {e_bt:.2e}")
    assert e_b <= BACK_TOL and e_s <= BACK_TOL and worst <= FWD_TOL and e_bt <= BACK_TOL


def test_osem_with_additive_term_and_empty_rays():
    """The fused ratio g / (H f + s) with a non-zero additive term s, from a
    start image whose lowest axial rows are zero so that those rows of every
    projection have H f = 0; s is 0 there too, so the ratio takes the R12
    branch (0 where H f + s <= 0).  Whole reconstruction and the stepwise
    driver against the oracle's OSEM with the same s and start image."""
    n, nz, A, M = 40, 24, 12, 4
    og, plan = both(n, nz, A, angles=list(np.random.default_rng(3).uniform(0, 360, A)))
    r = np.random.default_rng(21)
    mu = P.random_mu(og.object_shape, r, 0.12)
    mu64 = mu.astype(np.float64)
    f_true = P.random_object(og.object_shape, r)
    s_add = (0.05 * P.random_object(og.proj_shape, r)).astype(np.float32)
    s_add[:, :, :6] = 0.0
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu64) + s_add, 3e5, r)
    f0 = (0.5 + P.random_object(og.object_shape, r)).astype(np.float32)
    f0[:, :, :14] = 0.0
    hf0 = O.forward(og, f0.astype(np.float64), mu64)
    assert not hf0[:, :, :6].any() and hf0[:, :, 6:].min() >= 0  # the R12 branch is reached
    ref = O.osem(og, g.astype(np.float64), mu64, 2, M, s=s_add.astype(np.float64), f0=f0.astype(np.float64))
    got = host(S.osem(plan, dev(g), 2, M, dev(mu), s_add=dev(s_add), f0=dev(f0)))
    got_s = host(S.osem_steps(plan, dev(g), 2, M, dev(mu), s_add=dev(s_add), f0=dev(f0)))
    e, e_s = rel_l2(got, ref), rel_l2(got_s, ref)
    say(f"  OSEM with s: whole {e:.2e}, stepwise {e_s:.2e}")
    assert e <= OSEM_TOL and e_s <= OSEM_TOL
    assert np.isfinite(got).all() and not got[:, :, :14].any()


def test_kernel_timer_counts_launches():
    og, plan = both(32, 16, 8)
    r = np.random.default_rng(15)
    f = dev(P.random_object(og.object_shape, r))
    mu = dev(P.random_mu(og.object_shape, r, 0.1))
    with S.KernelTimer() as kt:
        for _ in range(3):
            plan.forward(f, mu)
        torch.cuda.synchronize()
    st = kt.stats()
    assert st["fwd_main"][0] == 3 and st["fwd_main"][1] > 0
    assert st["fwd_reduce"][0] == 3
    plan.forward(f, mu)   # not recorded once the timer is closed
    torch.cuda.synchronize()
    assert kt.stats() == {}


def test_whole_reconstruction_matches_stepwise_driver():
    """osem_reconstruct (attenuation factors read from the subset's table)
    gives the image of spect_sensitivity + osem_subset_step driven from Python
    (mu resampled, its depth sums split at other chunk boundaries) to FP32
    rounding: each ray sums up to 128 depths in a different order, about
    sqrt(128) x 6e-8 = 7e-7 relative per projection, so the bar is 2e-6;
    uneven subsets (60 angles in 8 subsets) included."""
    w = P.C1
    og, f_true, mu, g = workload_data(P.C2)
    plan = S.Plan.for_workload(P.C2)
    gd, mud = dev(g), dev(mu)
    a = host(S.osem(plan, gd, 1, 8, mud))
    b = host(S.osem_steps(plan, gd, 1, 8, mud))
    e = rel_l2(a, b)
    say(f"  128^3 one iteration: reconstruct vs stepwise rel L2 {e:.2e}")
    assert e <= 2e-6
    r = np.random.default_rng(16)
    og2, plan2 = both(32, 24, 60)
    f2 = P.random_object(og2.object_shape, r) + 0.5
    mu2 = P.random_mu(og2.object_shape, r, 0.15)
    g2 = P.poisson_counts(O.forward(og2, f2.astype(np.float64), mu2.astype(np.float64)), 1e5, r)
    got = host(S.osem(plan2, dev(g2), 2, 8, dev(mu2)))
    ref = O.osem(og2, g2.astype(np.float64), mu2.astype(np.float64), 2, 8)
    e2 = rel_l2(got, ref)
    say(f"  uneven subsets (60 angles / 8): OSEM rel L2 {e2:.2e}")
    assert e2 <= OSEM_TOL
    assert w.n_subsets == 6


@pytest.mark.parametrize("n,nz,A,idx", [(37, 20, 12, [0, 3, 4, 11]), (16, 8, 130, None),
                                        (128, 128, 120, list(range(2, 120, 8)))])
def test_attenuation_table_calls_match_the_oracle(n, nz, A, idx):
    """spect_sensitivity_table writes the factors of the listed angles while it
    computes H^T 1; spect_fwd_table / spect_back_table read them.  All three
    against the oracle with the attenuation map (lists longer than one launch
    included: 130 angles), and against the map-based calls."""
    og, plan = both(n, nz, A)
    r = np.random.default_rng(50 + n)
    mu = P.random_mu(og.object_shape, r, 0.15)
    f = P.random_object(og.object_shape, r)
    y = P.random_object(og.proj_shape, r)
    mud = dev(mu)
    rows = list(range(A)) if idx is None else idx
    sens_t, table = plan.sensitivity_table(mud, idx)
    assert table.numel() * 4 == plan.table_size(len(rows))
    ref_s = O.back(og, np.ones(og.proj_shape), mu.astype(np.float64), rows)
    e_s = rel_l2(host(sens_t), ref_s)
    e_s2 = rel_l2(host(sens_t), host(plan.sensitivity(mud, idx)))
    fp = host(plan.forward_table(dev(f), table, idx))
    ref_f = O.forward(og, f.astype(np.float64), mu.astype(np.float64), rows)
    worst = max(rel_l2(fp[i], ref_f[i]) for i in rows)
    bp = host(plan.back_table(dev(y), table, idx))
    ref_b = O.back(og, y.astype(np.float64), mu.astype(np.float64), rows)
    e_b = rel_l2(bp, ref_b)
    say(f"  {n}x{n}x{nz}, {len(rows)} angles: sens {e_s:.2e} (vs map call {e_s2:.2e}), "
        f"forward worst {worst:.2e}, back {e_b:.2e}")
    assert e_s <= BACK_TOL and e_s2 <= 1e-6 and worst <= FWD_TOL and e_b <= BACK_TOL
    others = np.setdiff1d(np.arange(A), rows)
    assert not fp[others].any()
    with pytest.raises(S.SpectError):
        plan.workspace_size(S.OP_OSEM, 2, 2)


@pytest.mark.parametrize("n,nz,A,M,orbit", [(32, 24, 30, 4, False), (40, 20, 13, 13, False),
                                             (24, 16, 12, 1, False), (32, 24, 30, 4, True)])
def test_reconstruction_without_attenuation_matches_per_subset_passes(n, nz, A, M, orbit):
    """Without an attenuation map osem_reconstruct runs the sensitivity pass
    of every subset as one launch over all angles (subset after subset) and
    the subsets' gathers as one launch; with one detector distance for every
    angle (the same blur taps) the pass forms one angle's brick, which the
    gathers read for every angle.  The sensitivities are the same values as
    the per-subset passes of spect_sensitivity, formed in the same order, so
    the reconstruction equals the stepwise driver's bitwise (uneven and
    one-angle subsets, a single subset, which takes the per-subset path, and a
    per-angle detector distance, which keeps a brick per angle).  Both meet
    the oracle's OSEM (Eq. 5)."""
    r = np.random.default_rng(1977 + n + A)
    rad = list(0.5 * n * 0.48 + 2.0 + 1.5 * np.cos(np.arange(A) * 2 * np.pi / A) ** 2) if orbit else None
    og, plan = both(n, nz, A, radius=rad)
    f = P.random_object(og.object_shape, r) + 0.5
    g = P.poisson_counts(O.forward(og, f.astype(np.float64), None), 1e5, r)
    gd = dev(g)
    a = host(S.osem(plan, gd, 2, M, None))
    b = host(S.osem_steps(plan, gd, 2, M, None))
    say(f"  {n}x{n}x{nz}, {A} angles / {M}: reconstruct vs stepwise rel L2 {rel_l2(a, b):.2e}")
    assert rel_l2(a, b) == 0.0
    ref = O.osem(og, g.astype(np.float64), None, 2, M)
    assert rel_l2(a, ref) <= OSEM_TOL
