"""The allocation-free forward projection (spect_fwd_static) on the GPU.

spect_fwd_static computes what spect_fwd does with the library's fixed
device scratch array instead of a caller workspace; through the C ABI its
projections must equal spect_fwd's on the same inputs (the same kernels and
launch split: bitwise, which is stricter than the 1e-5 projection bar), on
two calls in a row with the second smaller than the first, listed rows only.
A launch whose scratch need exceeds the array is refused before any launch.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

from oracle import oracle as O
import paper_2309_01977_amd as S
from paper_2309_01977_amd import _binding as B
from paper_2309_01977_amd import phantoms as P

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    O.build(force=False)
    S.load_library()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def static_call(plan, f, mu, idx, out):
    lib = S.load_library()
    arr = (ctypes.c_int32 * len(idx))(*idx)
    st = lib.spect_fwd_static(plan._h, ctypes.c_void_p(f.data_ptr()),
                              None if mu is None else ctypes.c_void_p(mu.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), arr, len(idx),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def test_static_scratch_forward_equals_the_workspace_forward_twice():
    cases = [(128, 128, 120, True, list(range(1, 120, 4))),   # the 128^3 geometry, 30 angles
             (40, 20, 12, True, [0, 3, 5, 6, 7, 9, 11]),       # then a smaller one
             (24, 6, 5, False, [4, 1])]                        # scalar path, no attenuation
    for n, nz, A, with_mu, idx in cases:
        say(f"  spect_fwd_static n={n} nz={nz} A={A} angles={len(idx)} mu={with_mu}")
        r = np.random.default_rng(900 + n)
        plan = S.Plan(n, nz, A, 0.48, 0.03, 0.1)
        need = plan.workspace_size(S.OP_FWD, len(idx), with_mu)
        assert need <= STATIC_BYTES
        f = dev(P.random_object(plan.object_shape, r))
        mu = dev(P.random_mu(plan.object_shape, r, 0.15)) if with_mu else None
        ref = plan.forward(f, mu, idx)
        out = torch.full(plan.proj_shape, -1.0, device="cuda")
        assert static_call(plan, f, mu, idx, out) == B.SPECT_OK, S.load_library().spect_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out[idx], ref[idx])
        rest = [a for a in range(A) if a not in idx]
        assert bool((out[rest] == -1.0).all())
        if n <= 40:
            og = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
            ro = O.forward(og, f.cpu().double().numpy(), None if mu is None else mu.cpu().double().numpy(), idx)
            got = out.cpu().double().numpy()
            worst = max(np.linalg.norm(got[a] - ro[a]) / np.linalg.norm(ro[a]) for a in idx)
            say(f"    vs oracle: worst per-projection rel L2 {worst:.2e}")
            assert worst <= 1e-5


def test_static_scratch_refuses_a_launch_beyond_its_size():
    plan = S.Plan(256, 256, 128, 0.48, 0.03, 0.1)
    idx = list(range(128))
    assert plan.workspace_size(S.OP_FWD, len(idx), True) > STATIC_BYTES
    f = torch.zeros(plan.object_shape, device="cuda")
    mu = torch.zeros(plan.object_shape, device="cuda")
    out = torch.full(plan.proj_shape, -1.0, device="cuda")
    assert static_call(plan, f, mu, idx, out) == B.SPECT_EINVAL
    assert "static scratch" in S.load_library().spect_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == -1.0).all())
