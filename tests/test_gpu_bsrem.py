"""BSREM with the relative difference prior on the GPU, through the C ABI,
against the FP64 oracle.

Bar: the prior gradient within 1e-5 relative L2 (an elementwise stencil in
FP32 against FP64); reconstructions within 1e-4 relative L2 after the run
(the OSEM bar).  Measured data are oracle projections of seeded phantoms.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import phantoms as P

pytestmark = pytest.mark.gpu

PRIOR_TOL = 1e-5
RECON_TOL = 1e-4
BETA, GAMMA = P.RDP_BETA, P.RDP_GAMMA


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


@pytest.mark.parametrize("shape", [(37, 37, 20), (16, 16, 5), (1, 1, 3)])
def test_prior_gradient_matches_the_oracle(shape):
    """Random non-negative images with a block of exact zeros (pairs with a
    zero denominator) and ragged sizes."""
    n, _, nz = shape
    plan = S.Plan(n, nz, 4, 0.48)
    r = np.random.default_rng(60 + n)
    f = P.random_object(shape, r)
    f[: n // 3, : n // 3, :] = 0.0
    for gamma in (GAMMA, 0.0):
        got = host(plan.rdp_gradient(dev(f), gamma))
        ref = O.rdp_gradient(f.astype(np.float64), gamma)
        assert np.isfinite(got).all()
        e = rel_l2(got, ref)
        say(f"  {shape} gamma {gamma}: prior gradient rel L2 {e:.2e}")
        assert e <= PRIOR_TOL


def test_prior_gradient_of_the_128cube_phantom():
    w = P.C6
    f, _ = P.make_phantom(w, ss=2)
    plan = S.Plan.for_workload(w)
    got = host(plan.rdp_gradient(dev(f), GAMMA))
    e = rel_l2(got, O.rdp_gradient(f.astype(np.float64), GAMMA))
    say(f"  128^3 phantom: prior gradient rel L2 {e:.2e}")
    assert e <= PRIOR_TOL


def small_problem(seed, n=32, nz=24, A=24):
    r = np.random.default_rng(seed)
    og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
    plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
    f_true = P.random_object(og.object_shape, r) + 0.2
    mu = P.random_mu(og.object_shape, r, 0.15)
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu.astype(np.float64)), 2e5, r)
    return og, plan, mu, g


def test_bsrem_many_iterations_matches_the_oracle():
    """10 iterations x 4 subsets with an explicit relaxation sequence, and the
    default sequence, against the oracle."""
    og, plan, mu, g = small_problem(61)
    relax = [1.0 / (1.0 + 0.5 * k) for k in range(10)]
    for rel in (relax, None):
        got = host(plan.bsrem(dev(g), 10, 4, dev(mu), beta=BETA, gamma=GAMMA, relaxation=rel))
        ref = O.bsrem(og, g.astype(np.float64), mu.astype(np.float64), 10, 4, BETA, GAMMA,
                      relaxation=None if rel is None else (lambda k: relax[k]))
        e = rel_l2(got, ref)
        say(f"  relaxation {'given' if rel else 'default'}: BSREM rel L2 {e:.2e}")
        assert e <= RECON_TOL


def test_bsrem_stepwise_driver_equals_whole_reconstruction():
    og, plan, mu, g = small_problem(62)
    M, I = 4, 3
    gd, mud = dev(g), dev(mu)
    whole = host(plan.bsrem(gd, I, M, mud, beta=BETA, gamma=GAMMA))
    sens = [plan.sensitivity(mud, S.subset_angles(og.n_angles, M, m)) for m in range(M)]
    sens_all = plan.sensitivity(mud)
    f = torch.ones(og.object_shape, device="cuda")
    for k in range(I):
        for m in range(M):
            plan.bsrem_subset_step(f, gd, sens[m], sens_all, m, M, 1.0 / (1.0 + k), BETA, GAMMA, mud)
    e = rel_l2(host(f), whole)
    say(f"  stepwise vs whole: rel L2 {e:.2e}")
    assert e <= 1e-5


@pytest.mark.timeout(900)
def test_bsrem_at_128cube_matches_the_oracle():
    """The benchmark geometry and data (128^3, 120 angles, attenuation, 8
    subsets), 2 iterations of BSREM-RDP with beta 0.3, gamma 2."""
    w = P.C6
    og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
    f_true, mu = P.make_phantom(w)
    _, noise = P.rngs(w.seed_index)
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu.astype(np.float64)), w.total_counts, noise)
    plan = S.Plan.for_workload(w)
    got = host(plan.bsrem(dev(g), 2, w.n_subsets, dev(mu), beta=BETA, gamma=GAMMA))
    say("  GPU BSREM done; running the oracle")
    ref = O.bsrem(og, g.astype(np.float64), mu.astype(np.float64), 2, w.n_subsets, BETA, GAMMA)
    e = rel_l2(got, ref)
    say(f"  128^3 BSREM-RDP 2 it x 8 subsets: rel L2 {e:.2e}")
    assert e <= RECON_TOL
    assert (got >= 0).all()
