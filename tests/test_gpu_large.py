"""Parity with the FP64 oracle at the large geometries.

The serving and batched workloads include a 192 x 192 x 160 grid with 128
angles, attenuation and the depth-dependent blur: its far depths need a
blur radius of 24 pixels (the 24-pixel blur class of the kernels), and a
224-wide grid reaches the 28-pixel class.  Bars as everywhere: forward
projections within 1e-5 relative L2 per projection, back projections and
sensitivities within 1e-5 over the volume, reconstructions within 1e-4.
"""
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
LARGE_ITERS, LARGE_SUBSETS = 2, 8


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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def blur_class(og):
    k = len(O.psf_taps(og, 0)) - 1
    return k, (k + 3) // 4 * 4


_CACHE = {}


def large():
    """The 192 x 192 x 160 x 128 workload: torso phantom and mu map, oracle
    data, and the oracle's OSEM of it (computed once for the module)."""
    if "w" not in _CACHE:
        w = P.C5_LARGE
        say(f"  building {w.name}: phantom, oracle projection")
        f_true, mu = P.make_phantom(w, ss=2)
        og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
        gbar = O.forward(og, f_true.astype(np.float64), mu.astype(np.float64))
        _, noise = P.rngs(w.seed_index)
        g = P.poisson_counts(gbar, w.total_counts, noise)
        _CACHE["w"] = (w, og, f_true, mu, gbar, g)
    return _CACHE["w"]


def large_osem_ref():
    if "osem" not in _CACHE:
        w, og, f_true, mu, gbar, g = large()
        say(f"  oracle OSEM {LARGE_ITERS} it x {LARGE_SUBSETS} subsets at {og.object_shape} x {og.n_angles}")
        _CACHE["osem"] = O.osem(og, g.astype(np.float64), mu.astype(np.float64), LARGE_ITERS, LARGE_SUBSETS)
    return _CACHE["osem"]


@pytest.mark.timeout(900)
def test_192_grid_projections_back_projection_and_sensitivity():
    w, og, f_true, mu, gbar, g = large()
    k, cls = blur_class(og)
    say(f"  blur radius at the far depth {k}, class {cls}")
    assert cls == 24
    plan = S.Plan.for_workload(w)
    mud, mu64 = dev(mu), mu.astype(np.float64)
    # every projection of the phantom (mu sampled in the kernels)
    got = host(plan.forward(dev(f_true), mud))
    worst = max(rel_l2(got[n], gbar[n]) for n in range(w.n_angles))
    say(f"  forward, all {w.n_angles} angles: worst per-projection rel L2 {worst:.2e}")
    assert worst <= FWD_TOL
    # back projection and sensitivity of one subset
    idx = list(range(3, w.n_angles, LARGE_SUBSETS))
    r = np.random.default_rng(190)
    y = P.random_object(og.proj_shape, r)
    e_b = rel_l2(host(plan.back(dev(y), mud, idx)), O.back(og, y.astype(np.float64), mu64, idx))
    ones_ref = O.back(og, np.ones(og.proj_shape), mu64, idx)
    e_s = rel_l2(host(plan.sensitivity(mud, idx)), ones_ref)
    say(f"  subset of {len(idx)} angles: back {e_b:.2e}, sensitivity {e_s:.2e}")
    assert e_b <= BACK_TOL and e_s <= BACK_TOL
    # the attenuation-table calls on the same subset
    sens_t, table = plan.sensitivity_table(mud, idx)
    e_st = rel_l2(host(sens_t), ones_ref)
    f = P.random_object(og.object_shape, r)
    fp = host(plan.forward_table(dev(f), table, idx))
    ref_f = O.forward(og, f.astype(np.float64), mu64, idx)
    worst_t = max(rel_l2(fp[i], ref_f[i]) for i in idx)
    e_bt = rel_l2(host(plan.back_table(dev(y), table, idx)), O.back(og, y.astype(np.float64), mu64, idx))
    say(f"  table calls: sensitivity {e_st:.2e}, forward worst {worst_t:.2e}, back {e_bt:.2e}")
    assert e_st <= BACK_TOL and worst_t <= FWD_TOL and e_bt <= BACK_TOL


@pytest.mark.timeout(900)
def test_192_grid_osem_reconstruction():
    """osem_reconstruct at 192 x 192 x 160 x 128 (2 it x 8 subsets, the
    attenuation tables of every subset in use) against the oracle's OSEM."""
    w, og, f_true, mu, gbar, g = large()
    plan = S.Plan.for_workload(w)
    got = host(S.osem(plan, dev(g), LARGE_ITERS, LARGE_SUBSETS, dev(mu)))
    e = rel_l2(got, large_osem_ref())
    say(f"  OSEM rel L2 {e:.2e}")
    assert e <= OSEM_TOL


@pytest.mark.timeout(900)
def test_batch_with_a_192_member_matches_the_oracle():
    """A batch holding the 192 x 192 x 160 x 128 reconstruction and a
    64^3 x 60 one: both members against the oracle, and bitwise against
    their own osem_reconstruct."""
    w, og, f_true, mu, gbar, g = large()
    r = np.random.default_rng(191)
    og2 = O.Geometry(64, 64, 60, 0.48, 0.03, 0.1)
    f2 = P.random_object(og2.object_shape, r) + 0.2
    mu2 = P.random_mu(og2.object_shape, r, 0.15)
    g2 = P.poisson_counts(O.forward(og2, f2.astype(np.float64), mu2.astype(np.float64)), 1e6, r)
    plans = [S.Plan.for_workload(w), S.Plan(64, 64, 60, 0.48, 0.03, 0.1)]
    batch = S.Batch(plans, LARGE_SUBSETS, True)
    fs = [torch.ones(p.object_shape, device="cuda") for p in plans]
    batch.reconstruct(fs, [dev(mu), dev(mu2)], [dev(g), dev(g2)], LARGE_ITERS)
    ref2 = O.osem(og2, g2.astype(np.float64), mu2.astype(np.float64), LARGE_ITERS, LARGE_SUBSETS)
    e1, e2 = rel_l2(host(fs[0]), large_osem_ref()), rel_l2(host(fs[1]), ref2)
    single = [host(S.osem(plans[0], dev(g), LARGE_ITERS, LARGE_SUBSETS, dev(mu))),
              host(S.osem(plans[1], dev(g2), LARGE_ITERS, LARGE_SUBSETS, dev(mu2)))]
    say(f"  batch members vs oracle: 192 {e1:.2e}, 64 {e2:.2e}")
    assert e1 <= OSEM_TOL and e2 <= OSEM_TOL
    np.testing.assert_array_equal(host(fs[0]), single[0])
    np.testing.assert_array_equal(host(fs[1]), single[1])


@pytest.mark.timeout(600)
def test_224_grid_reaches_the_28_pixel_blur_class():
    n, nz, A = 224, 24, 4
    og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1, 4.0, [0.0, 41.0, 137.0, 300.0])
    plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1, 4.0, [0.0, 41.0, 137.0, 300.0])
    k, cls = blur_class(og)
    say(f"  blur radius at the far depth {k}, class {cls}")
    assert cls == 28
    r = np.random.default_rng(224)
    f = P.random_object(og.object_shape, r)
    mu = P.random_mu(og.object_shape, r, 0.05)
    mu64 = mu.astype(np.float64)
    ref = O.forward(og, f.astype(np.float64), mu64)
    got = host(plan.forward(dev(f), dev(mu)))
    worst = max(rel_l2(got[i], ref[i]) for i in range(A))
    y = P.random_object(og.proj_shape, r)
    e_b = rel_l2(host(plan.back(dev(y), dev(mu))), O.back(og, y.astype(np.float64), mu64))
    idx = [1, 3]
    sens_t, table = plan.sensitivity_table(dev(mu), idx)
    e_s = rel_l2(host(sens_t), O.back(og, np.ones(og.proj_shape), mu64, idx))
    fp = host(plan.forward_table(dev(f), table, idx))
    worst_t = max(rel_l2(fp[i], ref[i]) for i in idx)
    say(f"  forward worst {worst:.2e}, back {e_b:.2e}, table: sens {e_s:.2e}, forward {worst_t:.2e}")
    assert worst <= FWD_TOL and e_b <= BACK_TOL and e_s <= BACK_TOL and worst_t <= FWD_TOL
    g = P.poisson_counts(ref, 2e5, r)
    e_o = rel_l2(host(S.osem(plan, dev(g), 1, 2, dev(mu))), O.osem(og, g.astype(np.float64), mu64, 1, 2))
    say(f"  OSEM 1 x 2 rel L2 {e_o:.2e}")
    assert e_o <= OSEM_TOL


@pytest.mark.timeout(600)
def test_192_grid_without_attenuation_shares_one_sensitivity_brick():
    """Without attenuation and with one detector distance for every angle,
    osem_reconstruct forms the constant projection's rotated-frame brick once
    and its subset gathers read it for every angle, also here, where a brick
    per angle (128 x 23.6 MB) would not fit the 512 MiB that form is limited
    to.  The reconstruction equals the stepwise driver's (spect_sensitivity
    per subset, a brick per angle) bitwise."""
    n, nz, A, M = 192, 160, 128, 8
    plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
    r = np.random.default_rng(192160)
    g = r.poisson(20.0, size=plan.proj_shape).astype(np.float32)
    gd = dev(g)
    a = host(S.osem(plan, gd, 1, M, None))
    b = host(S.osem_steps(plan, gd, 1, M, None))
    say(f"  {n}x{n}x{nz}, {A} angles / {M}: reconstruct vs stepwise max |diff| {np.abs(a - b).max():.2e}")
    assert np.isfinite(a).all() and a.max() > 0
    np.testing.assert_array_equal(a, b)
