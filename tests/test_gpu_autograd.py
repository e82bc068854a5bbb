"""The projector pair as autograd Functions, and unrolled OSEM, on the GPU.

Checks, through the C ABI: the gradient of a projection is the oracle's
transpose (and the gradient of a back projection its forward projection);
the gradient of the loss of 10 unrolled OSEM subiterations with respect to
the initial image matches the FP64 oracle's reverse recursion and central
finite differences (eps 1e-3); checkpointing and batching change nothing; the
fused subiteration over an angle list (osem_list_step) equals the subset
subiteration bitwise and the oracle's step, and its vector-Jacobian product
(osem_list_step_vjp) matches the oracle's reverse step and central
differences; invalid lists are refused.
Bar: projections within 1e-5 relative L2 (the projector bar); the unrolled
loss and its gradient within 1e-4 relative L2 (the OSEM bar: the gradient
applies the same FP32 projectors as the OSEM run, twice as often).
Inputs are seeded; measured data are oracle projections of the phantoms.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import phantoms as P

pytestmark = pytest.mark.gpu

PROJ_TOL = 1e-5
GRAD_TOL = 1e-4


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


def small_problem(seed, n=32, nz=24, A=24, with_s=False):
    r = np.random.default_rng(seed)
    og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
    plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
    f_true = P.random_object(og.object_shape, r) + 0.2
    mu = P.random_mu(og.object_shape, r, 0.15)
    g = P.poisson_counts(O.forward(og, f_true.astype(np.float64), mu.astype(np.float64)), 2e5, r)
    s = (0.05 * r.random(og.proj_shape)).astype(np.float32) if with_s else None
    return og, plan, f_true, mu, g, s


def test_gradients_of_the_projector_pair_are_the_oracle_transposes():
    og, plan, f_true, mu, _, _ = small_problem(40)
    r = np.random.default_rng(41)
    idx = [1, 5, 6, 17, 23]
    y = P.random_object(og.proj_shape, r, signed=True)
    f = dev(f_true).requires_grad_(True)
    (S.project(f, plan, dev(mu), idx) * dev(y)).sum().backward()
    ref = O.back(og, y.astype(np.float64), mu.astype(np.float64), idx)
    e = rel_l2(host(f.grad), ref)
    say(f"  d<Hf,y>/df vs oracle H^T y: rel L2 {e:.2e}")
    assert e <= PROJ_TOL
    x = P.random_object(og.object_shape, r, signed=True)
    p = dev(y).requires_grad_(True)
    (S.back_project(p, plan, dev(mu), idx) * dev(x)).sum().backward()
    refp = O.forward(og, x.astype(np.float64), mu.astype(np.float64), idx)
    gp = host(p.grad)
    e2 = rel_l2(gp[idx], refp[idx])
    say(f"  d<H^T p,x>/dp vs oracle H x: rel L2 {e2:.2e}")
    assert e2 <= PROJ_TOL
    others = np.setdiff1d(np.arange(og.n_angles), idx)
    assert not gp[others].any()


@pytest.mark.parametrize("with_s", [False, True])
def test_unrolled_osem_gradient_matches_the_oracle(with_s):
    og, plan, f_true, mu, g, s = small_problem(42, with_s=with_s)
    K, M = 10, 4
    f0 = np.ones(og.object_shape, np.float32)
    loss_ref, grad_ref = O.unrolled_osem_grad(og, g.astype(np.float64), f0.astype(np.float64),
                                              f_true.astype(np.float64), K, M, mu.astype(np.float64),
                                              None if s is None else s.astype(np.float64))
    f = dev(f0).requires_grad_(True)
    fk = S.unrolled_osem(plan, dev(g), f, K, M, dev(mu), None if s is None else dev(s))
    loss = ((fk.double() - dev(f_true).double()) ** 2).mean()
    loss.backward()
    el = abs(loss.item() - loss_ref) / loss_ref
    eg = rel_l2(host(f.grad), grad_ref)
    say(f"  s={'yes' if with_s else 'no'}: loss rel err {el:.2e}, gradient rel L2 {eg:.2e}")
    assert el <= GRAD_TOL and eg <= GRAD_TOL


def test_attenuation_tables_give_the_same_gradient():
    """Unrolled OSEM reading per-subset attenuation tables (written by the
    sensitivity pass) against the oracle, and against the map-based run."""
    og, plan, f_true, mu, g, _ = small_problem(47)
    K, M = 10, 4
    mud = dev(mu)
    sens, tables = S.autograd.subset_sensitivities(plan, M, mud, tables=True)
    grads = []
    for tabs in (tables, None):
        f = torch.ones(og.object_shape, device="cuda", requires_grad=True)
        fk = S.unrolled_osem(plan, dev(g), f, K, M, mud, sens=sens, tables=tabs)
        ((fk.double() - dev(f_true).double()) ** 2).mean().backward()
        grads.append(host(f.grad))
    _, grad_ref = O.unrolled_osem_grad(og, g.astype(np.float64), np.ones(og.object_shape),
                                       f_true.astype(np.float64), K, M, mu.astype(np.float64))
    e_ref, e_map = rel_l2(grads[0], grad_ref), rel_l2(grads[0], grads[1])
    say(f"  tables: gradient rel L2 {e_ref:.2e} vs oracle, {e_map:.2e} vs map-based run")
    assert e_ref <= GRAD_TOL and e_map <= 1e-5


def test_unrolled_osem_gradient_matches_central_differences():
    og, plan, f_true, mu, g, _ = small_problem(43)
    K, M = 10, 4
    gd, mud, td = dev(g), dev(mu), dev(f_true).double()
    sens = S.autograd.subset_sensitivities(plan, M, mud)

    def loss_of(f0):
        fk = S.unrolled_osem(plan, gd, f0, K, M, mud, sens=sens, checkpointing=False)
        return ((fk.double() - td) ** 2).mean()

    f = torch.ones(og.object_shape, device="cuda", requires_grad=True)
    loss_of(f).backward()
    grad = f.grad.double()
    r = np.random.default_rng(44)
    eps = 1e-3
    for t in range(3):
        v = dev(r.standard_normal(og.object_shape))
        with torch.no_grad():
            fd = (loss_of(1.0 + eps * v) - loss_of(1.0 - eps * v)).item() / (2 * eps)
        an = (grad * v.double()).sum().item()
        say(f"  direction {t}: central difference {fd:.6e}, autograd {an:.6e}")
        assert abs(fd - an) <= 1e-2 * abs(an)


def test_checkpointing_and_batching_do_not_change_the_gradient():
    og, plan, f_true, mu, g, _ = small_problem(45)
    r = np.random.default_rng(46)
    B, K, M = 3, 6, 4
    f0 = np.stack([np.ones(og.object_shape, np.float32) + 0.1 * b for b in range(B)])
    gs = np.stack([g * (1 + 0.2 * b) for b in range(B)]).astype(np.float32)
    mus = np.stack([mu * (1 + 0.1 * b) for b in range(B)]).astype(np.float32)
    tgt = np.stack([P.random_object(og.object_shape, r) for _ in range(B)])
    grads = []
    for ck in (True, False):
        f = dev(f0).requires_grad_(True)
        fk = S.unrolled_osem(plan, dev(gs), f, K, M, dev(mus), checkpointing=ck)
        ((fk - dev(tgt)) ** 2).sum().backward()
        grads.append(host(f.grad))
    np.testing.assert_array_equal(grads[0], grads[1])
    f1 = dev(f0[1]).requires_grad_(True)
    fk1 = S.unrolled_osem(plan, dev(gs[1]), f1, K, M, dev(mus[1]))
    ((fk1 - dev(tgt[1])) ** 2).sum().backward()
    np.testing.assert_array_equal(host(f1.grad), grads[0][1])


@pytest.mark.timeout(900)
def test_batch_of_eight_at_128cube_matches_the_oracle():
    """The differentiable workload at full size, as bench.py runs it: 8 torso
    phantoms at 128^3 with 120 angles, 10 unrolled subiterations (8 subsets)
    with checkpointing and per-subset attenuation tables, loss = mean squared
    error to the phantoms; member 0's loss and gradient against the FP64
    oracle."""
    w, B, K = P.C4, P.C4_BATCH, P.C4_STEPS
    og = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b, w.psf_nsigma)
    plan = S.Plan.for_workload(w)
    f_true, mu = P.make_phantom_batch(w, B, ss=2)
    _, noise = P.rngs(w.seed_index)
    g = np.stack([P.poisson_counts(O.forward(og, f_true[b].astype(np.float64), mu[b].astype(np.float64)),
                                   w.total_counts, noise) for b in range(B)])
    say("  oracle data ready")
    f = torch.ones((B,) + w.object_shape, device="cuda", requires_grad=True)
    mud = dev(mu)
    sens, tables = S.autograd.subset_sensitivities(plan, w.n_subsets, mud, tables=True)
    fk = S.unrolled_osem(plan, dev(g), f, K, w.n_subsets, mud, sens=sens, tables=tables)
    loss = ((fk.double() - dev(f_true).double()) ** 2).mean(dim=(1, 2, 3))
    loss.sum().backward()
    got_loss, got_grad = loss[0].item(), host(f.grad[0])
    say("  GPU batch done; oracle gradient of member 0")
    loss_ref, grad_ref = O.unrolled_osem_grad(og, g[0].astype(np.float64), np.ones(w.object_shape),
                                              f_true[0].astype(np.float64), K, w.n_subsets,
                                              mu[0].astype(np.float64))
    el = abs(got_loss - loss_ref) / loss_ref
    eg = rel_l2(got_grad, grad_ref)
    say(f"  member 0: loss rel err {el:.2e}, gradient rel L2 {eg:.2e}")
    assert el <= GRAD_TOL and eg <= GRAD_TOL
    assert np.isfinite(host(f.grad)).all()


def _oracle_step(og, f, g, mu, idx, s=None):
    """The oracle's OSEM subiteration over the angles idx (0/0 readings as in
    osem_list_step), composed from its forward and back projections."""
    ghat = O.forward(og, f, mu, idx)
    if s is not None:
        ghat[idx] += s[idx]
    q = np.zeros(og.proj_shape)
    rows = np.zeros(og.proj_shape, dtype=bool)
    rows[idx] = ghat[idx] > 0
    q[rows] = g[rows] / ghat[rows]
    b = O.back(og, q, mu, idx)
    sens = O.back(og, np.ones(og.proj_shape), mu, idx)
    out = f.copy()
    pos = sens > 0
    out[pos] = f[pos] * b[pos] / sens[pos]
    return out


@pytest.mark.parametrize("with_s", [False, True])
def test_list_step_equals_the_subset_step(with_s):
    og, plan, f_true, mu, g, s = small_problem(50, with_s=with_s)
    M, m = 4, 1
    idx = list(range(m, og.n_angles, M))
    mud, gd, sd = dev(mu), dev(g), None if s is None else dev(s)
    sens = plan.sensitivity(mud, idx)
    f0 = dev(f_true * 0.5 + 0.3)
    ref = f0.clone()
    plan.osem_subset_step(ref, gd, sens, m, M, mud, sd)
    out = plan.osem_list_step(f0, gd, sens, idx, mu=mud, s_add=sd)
    inplace = f0.clone()
    plan.osem_list_step(inplace, gd, sens, idx, mu=mud, s_add=sd, out=inplace)
    np.testing.assert_array_equal(host(out), host(ref))
    np.testing.assert_array_equal(host(inplace), host(ref))
    # the subset's attenuation table in place of the map
    sens_t, table = plan.sensitivity_table(mud, idx)
    out_t = plan.osem_list_step(f0, gd, sens_t, idx, table=table, s_add=sd)
    e = rel_l2(host(out_t), host(ref))
    say(f"  s={'yes' if with_s else 'no'}: table vs map {e:.2e}")
    assert e <= 1e-5


@pytest.mark.parametrize("variant", ["map", "map+s", "table", "none"])
def test_list_step_product_matches_the_oracle_reverse_step(variant):
    """One subiteration followed by the loss mean((f1 - target)^2): the
    product of osem_list_step_vjp with 2 (f1 - target) / n is the oracle's
    dL/df0 for n_steps = 1."""
    og, plan, f_true, mu, g, s = small_problem(51, with_s=variant == "map+s")
    M = 3
    idx = list(range(0, og.n_angles, M))
    mu_o = None if variant == "none" else mu.astype(np.float64)
    if variant == "none":
        g = P.poisson_counts(O.forward(og, f_true.astype(np.float64)), 2e5, np.random.default_rng(52))
    r = np.random.default_rng(53)
    f0 = (P.random_object(og.object_shape, r) + 0.5).astype(np.float32)
    loss_ref, grad_ref = O.unrolled_osem_grad(og, g.astype(np.float64), f0.astype(np.float64),
                                              f_true.astype(np.float64), 1, M, mu_o,
                                              None if s is None else s.astype(np.float64))
    mud = None if variant == "none" else dev(mu)
    gd, sd = dev(g), None if s is None else dev(s)
    kw = dict(mu=mud, s_add=sd)
    if variant == "table":
        sens, table = plan.sensitivity_table(mud, idx)
        kw = dict(table=table)
    else:
        sens = plan.sensitivity(mud, idx)
    fd = dev(f0)
    f1 = plan.osem_list_step(fd, gd, sens, idx, **kw)
    gout = 2.0 * (f1 - dev(f_true)) / f1.numel()
    grad = plan.osem_list_step_vjp(fd, gd, sens, idx, gout, **kw)
    # the gradient may overwrite grad_out
    grad2 = plan.osem_list_step_vjp(fd, gd, sens, idx, gout, out=gout, **kw)
    eg = rel_l2(host(grad), grad_ref)
    say(f"  {variant}: gradient rel L2 {eg:.2e}")
    assert eg <= GRAD_TOL
    np.testing.assert_array_equal(host(grad2), host(grad))


def test_list_step_on_an_arbitrary_list_matches_the_oracle_and_central_differences():
    og, plan, f_true, mu, g, s = small_problem(54, with_s=True)
    idx = [2, 3, 9, 10, 11, 19]
    mud, gd, sd = dev(mu), dev(g), dev(s)
    sens = plan.sensitivity(mud, idx)
    r = np.random.default_rng(55)
    f0 = (P.random_object(og.object_shape, r) + 0.5).astype(np.float32)
    out = plan.osem_list_step(dev(f0), gd, sens, idx, mu=mud, s_add=sd)
    ref = _oracle_step(og, f0.astype(np.float64), g.astype(np.float64), mu.astype(np.float64), idx,
                       s.astype(np.float64))
    e = rel_l2(host(out), ref)
    say(f"  step vs oracle: {e:.2e}")
    assert e <= GRAD_TOL
    w = dev(r.standard_normal(og.object_shape))
    grad = plan.osem_list_step_vjp(dev(f0), gd, sens, idx, w, mu=mud, s_add=sd).double()
    eps = 1e-3
    for t in range(3):
        v = dev(r.standard_normal(og.object_shape))
        fp = plan.osem_list_step(dev(f0) + eps * v, gd, sens, idx, mu=mud, s_add=sd).double()
        fm = plan.osem_list_step(dev(f0) - eps * v, gd, sens, idx, mu=mud, s_add=sd).double()
        fdd = ((fp - fm) * w.double()).sum().item() / (2 * eps)
        an = (grad * v.double()).sum().item()
        say(f"  direction {t}: central difference {fdd:.6e}, product {an:.6e}")
        assert abs(fdd - an) <= 1e-2 * abs(an)


def test_list_step_refuses_invalid_lists():
    og, plan, f_true, mu, g, _ = small_problem(56)
    mud, gd, fd = dev(mu), dev(g), dev(f_true)
    sens = plan.sensitivity(mud, [0, 1])
    with pytest.raises(S.SpectError, match="listed twice"):
        plan.osem_list_step(fd, gd, sens, [0, 1, 0], mu=mud)
    with pytest.raises(S.SpectError, match="empty"):
        plan.osem_list_step(fd, gd, sens, [], mu=mud)
    _, table = plan.sensitivity_table(mud, [0, 1])
    with pytest.raises(ValueError, match="not both"):
        plan.osem_list_step(fd, gd, sens, [0, 1], mu=mud, table=table)
    big = S.Plan(8, 4, 130, 0.48)
    f8 = torch.ones(big.object_shape, device="cuda")
    g8 = torch.ones(big.proj_shape, device="cuda")
    with pytest.raises(S.SpectError, match="more than 128"):
        big.osem_list_step(f8, g8, f8, None)
