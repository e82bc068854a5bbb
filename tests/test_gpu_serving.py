"""The reconstruction server (spect_server_*) on the GPU.

Each result must be the same alone (osem_reconstruct on its own) and in the
mix (admitted while other requests are resident, every tick advancing all of
them together through shared launches): the bar is the OSEM bar, 1e-4
relative L2, and the server's steps use osem_reconstruct's arguments, so the
results are asserted bitwise; one request per class is also checked against
the FP64 oracle.  Admission follows the memory footprint; a short request
admitted beside a long one finishes first (iteration-level scheduling).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import phantoms as P
from paper_2309_01977_amd import serving

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


# (n, nz, angles, attenuation, iterations, subsets)
CLASSES = [(24, 16, 18, False, 2, 3), (32, 24, 24, True, 2, 4), (40, 20, 30, True, 1, 5)]


def make_classes(seed, per_class=3):
    r = np.random.default_rng(seed)
    out = []
    for n, nz, A, with_mu, I, M in CLASSES:
        og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
        plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
        gs, mus = [], []
        for _ in range(per_class):
            f = P.random_object(og.object_shape, r) + 0.2
            mu = P.random_mu(og.object_shape, r, 0.15) if with_mu else None
            g = P.poisson_counts(O.forward(og, f.astype(np.float64), None if mu is None else mu.astype(np.float64)),
                                 1e5, r)
            gs.append(g)
            mus.append(mu)
        out.append((og, plan, gs, mus if with_mu else None, I, M))
    return out


def alone(plan, g, mu, I, M, s=None):
    return host(S.osem(plan, dev(g), I, M, None if mu is None else dev(mu), None if s is None else dev(s)))


def footprint(plan, M, with_mu):
    return plan.workspace_size(S.OP_RECON, M, with_mu)


def test_results_are_the_same_alone_and_in_the_mix():
    """Nine mixed requests (class 1 with an additive term) on a 3-slot
    server: each result equals the same reconstruction run alone bitwise (the
    same kernels on the same data; overlap changes only the timing), and the
    oracle's OSEM within the OSEM bar."""
    cls = make_classes(80)
    r = np.random.default_rng(83)
    adds = {(1, k): (0.1 * P.random_object(cls[1][0].proj_shape, r)).astype(np.float32) for k in range(3)}
    server = S.Server(3, 1 << 30)
    jobs = []
    for k in range(3):
        for c, (og, plan, gs, mus, I, M) in enumerate(cls):
            f = torch.ones(plan.object_shape, device="cuda")
            mu = None if mus is None else dev(mus[k])
            s = adds.get((c, k))
            rid = server.submit(plan, f, dev(gs[k]), I, M, mu, None if s is None else dev(s))
            jobs.append((rid, c, k, f))
    for rid, *_ in jobs:
        server.wait(rid)
    running, queued, peak, used = server.stats()
    say(f"  {len(jobs)} requests, peak running {peak}")
    assert running == 0 and queued == 0 and used == 0 and peak >= 2
    for rid, c, k, f in jobs:
        og, plan, gs, mus, I, M = cls[c]
        mu = None if mus is None else mus[k]
        s = adds.get((c, k))
        got, ref = host(f), alone(plan, gs[k], mu, I, M, s)
        e = rel_l2(got, ref)
        assert e == 0.0, (c, k, e)
        if k == 0:
            eo = rel_l2(got, O.osem(og, gs[k].astype(np.float64), None if mu is None else mu.astype(np.float64),
                                    I, M, s=None if s is None else s.astype(np.float64)))
            say(f"  class {c}: in the mix vs alone {e:.2e}, vs oracle {eo:.2e}")
            assert eo <= OSEM_TOL
    server.close()


def test_admission_follows_the_memory_footprint():
    cls = make_classes(81, per_class=4)
    og, plan, gs, mus, I, M = cls[2]
    need = footprint(plan, M, True)
    for pool, expect_single in ((need + 4096, True), (4 * need + 4096, False)):
        server = S.Server(4, pool)
        fs, rids = [], []
        for k in range(4):
            f = torch.ones(plan.object_shape, device="cuda")
            rids.append(server.submit(plan, f, dev(gs[k]), I, M, dev(mus[k])))
            fs.append(f)
        for rid in rids:
            server.wait(rid)
        peak = server.stats()[2]
        say(f"  pool {pool} B for requests of {need} B: peak running {peak}")
        assert (peak == 1) if expect_single else (peak >= 2)
        for k, f in enumerate(fs):
            assert rel_l2(host(f), alone(plan, gs[k], mus[k], I, M)) <= OSEM_TOL
        server.close()


def test_a_request_larger_than_the_pool_is_refused():
    cls = make_classes(82, per_class=1)
    og, plan, gs, mus, I, M = cls[1]
    server = S.Server(2, footprint(plan, M, True) // 2)
    with pytest.raises(S.SpectError):
        server.submit(plan, torch.ones(plan.object_shape, device="cuda"), dev(gs[0]), I, M, dev(mus[0]))
    server.close()


def test_replayed_poisson_trace_completes_with_the_same_results():
    cls = make_classes(83)
    rcs = [serving.RequestClass(f"c{c}", plan, [dev(g) for g in gs], None if mus is None else [dev(m) for m in mus],
                                I, M) for c, (og, plan, gs, mus, I, M) in enumerate(cls)]
    trace = serving.poisson_trace(40.0, 1.0, len(rcs), np.random.default_rng(84))
    server = S.Server(4, 1 << 30)
    served = serving.replay(server, rcs, trace, keep_images=True)
    st = serving.summary(served)
    say(f"  {st['requests']} requests: p50 {st['latency_ms_p50']:.2f} ms, p99 {st['latency_ms_p99']:.2f} ms")
    assert st["requests"] == len(trace) and all(s.latency > 0 for s in served)
    for s in served[:8]:
        og, plan, gs, mus, I, M = cls[s.cls]
        mu = None if mus is None else mus[s.data_index]
        assert rel_l2(host(s.f), alone(plan, gs[s.data_index], mu, I, M)) <= OSEM_TOL
    server.close()


def test_requests_wait_for_inputs_written_on_the_callers_stream():
    """The initial image, the data and the attenuation map are written by
    work queued on the caller's (torch's) stream right before submission,
    behind a dozen milliseconds of other kernels; the request must be
    ordered after that work, so the result equals the reconstruction alone
    and not one of the placeholder values the arrays held before."""
    cls = make_classes(85, per_class=1)
    og, plan, gs, mus, I, M = cls[1]
    g_src, mu_src = dev(gs[0]), dev(mus[0])
    f = torch.full(plan.object_shape, 7.0, device="cuda")
    g = torch.full(plan.proj_shape, 1e6, device="cuda")
    mu = torch.full(plan.object_shape, 5.0, device="cuda")
    torch.cuda.synchronize()
    a = torch.randn(4096, 4096, device="cuda")
    for _ in range(12):
        a = torch.tanh(a @ a)
    f.fill_(1.0)
    g.copy_(g_src)
    mu.copy_(mu_src)
    server = S.Server(2, 1 << 30)
    rid = server.submit(plan, f, g, I, M, mu)
    server.wait(rid)
    got, ref = host(f), alone(plan, gs[0], mus[0], I, M)
    e = rel_l2(got, ref)
    say(f"  inputs written on the caller's stream: vs alone {e:.2e}")
    assert e == 0.0
    server.close()


def test_short_requests_finish_first_beside_long_ones():
    """A long reconstruction (3 iterations x 6 subsets at 40^2 x 20 with
    attenuation) and, submitted after it, short ones (1 x 3 at 24^2 x 16):
    all are resident together and every tick advances each of them by one
    step, so the short requests finish while the long one still runs; all
    results equal their reconstructions alone bitwise."""
    cls = make_classes(86, per_class=3)
    og_l, plan_l, gs_l, mus_l, _, _ = cls[2]
    og_s, plan_s, gs_s, _, _, _ = cls[0]
    server = S.Server(4, 1 << 30)
    g_long, mu_long = dev(gs_l[0]), dev(mus_l[0])
    g_short = [dev(g) for g in gs_s]
    f_long = torch.ones(plan_l.object_shape, device="cuda")
    fs = [torch.ones(plan_s.object_shape, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    # a dozen milliseconds of work on the caller's stream: every request's
    # first step waits for it, so all of them start together
    a = torch.randn(4096, 4096, device="cuda")
    for _ in range(12):
        a = torch.tanh(a @ a)
    rid_long = server.submit(plan_l, f_long, g_long, 3, 6, mu_long)
    shorts = [(server.submit(plan_s, fs[k], g_short[k], 1, 3), fs[k], k) for k in range(3)]
    states = []
    for rid, f, k in shorts:
        server.wait(rid)
        states.append(server.status(rid_long))
    server.wait(rid_long)
    peak = server.stats()[2]
    say(f"  long request's state as each short one finished: {states}, peak resident {peak}")
    assert peak == 4
    assert states[-1] == S.REQ_RUNNING
    for rid, f, k in shorts:
        assert rel_l2(host(f), alone(plan_s, gs_s[k], None, 1, 3)) == 0.0
    assert rel_l2(host(f_long), alone(plan_l, gs_l[0], mus_l[0], 3, 6)) == 0.0
    server.close()
