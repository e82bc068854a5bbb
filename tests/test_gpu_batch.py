"""Batched OSEM (spect_batch_*, osem_batch_reconstruct) on the GPU.

Every member of a batch must come out bitwise as its own osem_reconstruct
does (the same kernel bodies on the same tasks), and within the OSEM bar
(1e-4 relative L2) of the FP64 oracle.  Schedules 0-3, the eager path
and repeated graph replays (with other device work and synchronisation in
between, and with new arrays) give the same images bitwise; schedules 4-7
sum each ray over all depths at once instead of per depth chunk, which
changes only the FP32 rounding (checked to 1e-5, and against the oracle).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import phantoms as P

pytestmark = pytest.mark.gpu

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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


# uneven members: (n, nz, angles); 20 slices exercises a partial slab, 6 the scalar path
SHAPES = [(32, 24, 24), (48, 16, 30), (40, 20, 26), (24, 8, 16)]
SHAPES_SCALAR = [(32, 24, 24), (20, 6, 12)]


def members(shapes, with_mu, seed):
    r = np.random.default_rng(seed)
    out = []
    for n, nz, A in shapes:
        og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
        plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
        f = P.random_object(og.object_shape, r) + 0.2
        mu = P.random_mu(og.object_shape, r, 0.15) if with_mu else None
        g = P.poisson_counts(O.forward(og, f.astype(np.float64), None if mu is None else mu.astype(np.float64)),
                             2e5, r)
        out.append((og, plan, mu, g))
    return out


def run_batch(mem, M, I, with_mu, schedule=None, eager=False, batch=None):
    batch = batch or S.Batch([m[1] for m in mem], M, with_mu)
    if schedule is not None:
        batch.set_schedule(schedule)
    fs = [torch.ones(m[1].object_shape, device="cuda") for m in mem]
    mus = [dev(m[2]) for m in mem] if with_mu else None
    batch.reconstruct(fs, mus, [dev(m[3]) for m in mem], I, eager=eager)
    return [host(f) for f in fs], batch


@pytest.mark.parametrize("with_mu", [True, False])
def test_batch_members_equal_single_reconstructions_and_the_oracle(with_mu):
    M, I = 4, 2
    mem = members(SHAPES, with_mu, 70)
    got, _ = run_batch(mem, M, I, with_mu)
    for (og, plan, mu, g), fb in zip(mem, got):
        single = host(S.osem(plan, dev(g), I, M, None if mu is None else dev(mu)))
        ref = O.osem(og, g.astype(np.float64), None if mu is None else mu.astype(np.float64), I, M)
        e1, e2 = rel_l2(fb, single), rel_l2(fb, ref)
        say(f"  {og.object_shape} x {og.n_angles}: batch vs single {e1:.2e}, vs oracle {e2:.2e}")
        assert e1 == 0.0 and e2 <= OSEM_TOL


def test_batch_members_with_additive_terms():
    """Members with and without an additive term s in one batch: each equals
    its own osem_reconstruct with the same s bitwise, graph-replayed and
    eager, and the oracle's OSEM with that s within the OSEM bar."""
    M, I = 4, 2
    mem = members(SHAPES, True, 74)
    r = np.random.default_rng(75)
    ss = [(0.1 * P.random_object(og.proj_shape, r)).astype(np.float32) if k % 2 == 0 else None
          for k, (og, _, _, _) in enumerate(mem)]
    batch = S.Batch([m[1] for m in mem], M, True)
    for eager in (False, True):
        fs = [torch.ones(m[1].object_shape, device="cuda") for m in mem]
        batch.reconstruct(fs, [dev(m[2]) for m in mem], [dev(m[3]) for m in mem], I,
                          s_adds=[None if s is None else dev(s) for s in ss], eager=eager)
        for (og, plan, mu, g), s, f in zip(mem, ss, fs):
            fb = host(f)
            single = host(S.osem(plan, dev(g), I, M, dev(mu), s_add=None if s is None else dev(s)))
            ref = O.osem(og, g.astype(np.float64), mu.astype(np.float64), I, M,
                         s=None if s is None else s.astype(np.float64))
            e1, e2 = rel_l2(fb, single), rel_l2(fb, ref)
            say(f"  eager={eager} {og.object_shape} x {og.n_angles} s={s is not None}: "
                f"batch vs single {e1:.2e}, vs oracle {e2:.2e}")
            assert e1 == 0.0 and e2 <= OSEM_TOL


def test_every_schedule_and_the_eager_path_give_the_same_images():
    M, I = 4, 2
    mem = members(SHAPES, True, 71)
    ref, batch = run_batch(mem, M, I, True, eager=True)
    for sched in range(8):
        runs = []
        for eager in (False, True):
            got, _ = run_batch(mem, M, I, True, schedule=sched, eager=eager, batch=batch)
            runs.append(got)
            for a, b, (og, _, mu, g) in zip(got, ref, mem):
                if sched & 4:
                    # one running depth sum instead of per-chunk partials: FP32 rounding only
                    assert rel_l2(a, b) <= 1e-5
                    assert rel_l2(a, O.osem(og, g.astype(np.float64), mu.astype(np.float64), I, M)) <= OSEM_TOL
                else:
                    np.testing.assert_array_equal(a, b)
        for a, b in zip(*runs):
            np.testing.assert_array_equal(a, b)   # graph = eager within a schedule
        say(f"  schedule {sched}: graph and eager agree with the reference")


def test_graph_replays_between_other_work_and_with_new_arrays():
    """Replay the captured iteration several times with eager torch work and
    synchronisations in between, and again after switching to other arrays
    (the tables are rebuilt, the graph kept); each result against the eager
    path."""
    M, I = 4, 3
    mem = members(SHAPES, True, 72)
    ref, batch = run_batch(mem, M, I, True, eager=True)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2 + 1).sum().item()
        torch.cuda.synchronize()
        got, _ = run_batch(mem, M, I, True, batch=batch)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
        say(f"  replay round {rep}: equal")


def test_scalar_path_members():
    M, I = 3, 2
    mem = members(SHAPES_SCALAR, True, 73)
    got, _ = run_batch(mem, M, I, True)
    for (og, plan, mu, g), fb in zip(mem, got):
        ref = O.osem(og, g.astype(np.float64), mu.astype(np.float64), I, M)
        e = rel_l2(fb, ref)
        say(f"  {og.object_shape}: vs oracle {e:.2e}")
        assert e <= OSEM_TOL


def test_autotune_picks_a_timed_schedule_and_keeps_the_images():
    M, I = 4, 2
    mem = members(SHAPES, True, 74)
    batch = S.Batch([m[1] for m in mem], M, True)
    fs = [torch.ones(m[1].object_shape, device="cuda") for m in mem]
    mus = [dev(m[2]) for m in mem]
    gs = [dev(m[3]) for m in mem]
    sched, ms = batch.autotune(fs, mus, gs)
    say(f"  autotune: schedule {sched}, ms per iteration {['%.3f' % x for x in ms]}")
    assert 0 <= sched <= 7 and all(x > 0 for x in ms)
    assert ms[sched] == min(ms)
    for f in fs:
        assert torch.all(f == 1.0)
    batch.reconstruct(fs, mus, gs, I)
    ref, _ = run_batch(mem, M, I, True, eager=True)
    for f, b in zip(fs, ref):
        np.testing.assert_array_equal(host(f), b)


def test_graph_is_captured_again_when_the_arrays_lose_16_byte_alignment():
    """The same batch first with 16-byte aligned images (vector kernels),
    then with images that start 4 bytes into their storage (scalar kernels):
    the captured iteration must not replay the vector kernels on the
    unaligned arrays.  Both runs against the oracle and bitwise against the
    eager path on the same arrays."""
    M, I = 4, 2
    mem = members(SHAPES, True, 76)
    batch = S.Batch([m[1] for m in mem], M, True)
    mus = [dev(m[2]) for m in mem]
    gs = [dev(m[3]) for m in mem]
    refs = [O.osem(og, g.astype(np.float64), mu.astype(np.float64), I, M) for og, _, mu, g in mem]
    for offset in (0, 1):
        fs = []
        for m in mem:
            n = int(np.prod(m[1].object_shape))
            buf = torch.empty(n + 4, device="cuda")
            f = buf[offset:offset + n].view(m[1].object_shape)
            assert (f.data_ptr() % 16 == 0) == (offset == 0)
            f.fill_(1.0)
            fs.append(f)
        batch.reconstruct(fs, mus, gs, I)
        got = [host(f) for f in fs]
        for f in fs:
            f.fill_(1.0)
        batch.reconstruct(fs, mus, gs, I, eager=True)
        for a, f, ref, m in zip(got, fs, refs, mem):
            e = rel_l2(a, ref)
            say(f"  offset {4 * offset} B {m[0].object_shape}: vs oracle {e:.2e}")
            assert e <= OSEM_TOL
            np.testing.assert_array_equal(a, host(f))
