"""The projector pair as torch.autograd Functions, and unrolled OSEM.

The paper builds its projectors from PyTorch operations so that they can sit
inside learned reconstruction (Section 1; the PET example of Section 3.2 hands
a PyTorch network to its deep-image-prior algorithm).  Here the system matrix H (Section 2.1.1, Eq. 1) is the HIP
forward projection and its gradient is the hand-written exact adjoint H^T
(spect_back), and vice versa; nothing is differentiated through the kernels
by autograd itself.

    project(f, plan, mu, idx)       rows idx of H f        backward: H^T
    back_project(p, plan, mu, idx)  sum_n in idx H_n^T p   backward: H (rows idx)

Both accept one object (N, N, Nz) / projection set (A, N, Nz) or a batch
with a leading dimension B; mu is then (B, N, N, Nz) or a single map shared
by the batch, or None.  mu is not differentiated.

``unrolled_osem`` differentiates K OSEM subiterations (Eq. 5 with the Table 1
preconditioner, in the multiplicative form) with respect to the initial
image; each subiteration can be recomputed in the backward pass instead of
stored (torch.utils.checkpoint).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch
from torch.utils.checkpoint import checkpoint

from ._binding import Plan, subset_angles


def _members(x: torch.Tensor, rank: int):
    return [x] if x.dim() == rank else list(x.unbind(0))


def _mu_of(mu: Optional[torch.Tensor], b: int, batched: bool):
    if mu is None:
        return None
    if batched and mu.dim() == 4:
        return mu[b]
    return mu


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan: Plan, mu, idx):
        ctx.plan, ctx.idx = plan, idx
        ctx.has_mu = mu is not None
        if ctx.has_mu:
            ctx.save_for_backward(mu)
        batched = f.dim() == 4
        outs = []
        for b, fb in enumerate(_members(f.contiguous(), 3)):
            outs.append(plan.forward(fb, _mu_of(mu, b, batched), idx))
        return torch.stack(outs) if batched else outs[0]

    @staticmethod
    def backward(ctx, gp):
        mu = ctx.saved_tensors[0] if ctx.has_mu else None
        batched = gp.dim() == 4
        outs = []
        for b, gb in enumerate(_members(gp.contiguous(), 3)):
            outs.append(ctx.plan.back(gb, _mu_of(mu, b, batched), ctx.idx))
        return (torch.stack(outs) if batched else outs[0]), None, None, None


class _BackProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, plan: Plan, mu, idx):
        ctx.plan, ctx.idx = plan, idx
        ctx.has_mu = mu is not None
        if ctx.has_mu:
            ctx.save_for_backward(mu)
        batched = p.dim() == 4
        outs = []
        for b, pb in enumerate(_members(p.contiguous(), 3)):
            outs.append(plan.back(pb, _mu_of(mu, b, batched), idx))
        return torch.stack(outs) if batched else outs[0]

    @staticmethod
    def backward(ctx, gf):
        mu = ctx.saved_tensors[0] if ctx.has_mu else None
        batched = gf.dim() == 4
        outs = []
        for b, gb in enumerate(_members(gf.contiguous(), 3)):
            outs.append(ctx.plan.forward(gb, _mu_of(mu, b, batched), ctx.idx))
        return (torch.stack(outs) if batched else outs[0]), None, None, None


def project(f: torch.Tensor, plan: Plan, mu: Optional[torch.Tensor] = None,
            idx: Optional[Sequence[int]] = None) -> torch.Tensor:
    """Rows idx of H f (zeros elsewhere); differentiable in f."""
    return _Project.apply(f, plan, mu, None if idx is None else list(idx))


def back_project(p: torch.Tensor, plan: Plan, mu: Optional[torch.Tensor] = None,
                 idx: Optional[Sequence[int]] = None) -> torch.Tensor:
    """sum over n in idx of H_n^T p[n]; differentiable in p."""
    return _BackProject.apply(p, plan, mu, None if idx is None else list(idx))


def _safe_div(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """a / b where b > 0, else 0 (the 0/0 reading of the ratio)."""
    pos = b > 0
    return torch.where(pos, a / torch.where(pos, b, torch.ones_like(b)), torch.zeros_like(a))


def osem_update(f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, plan: Plan, idx,
                mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One OSEM subiteration on the angles idx, differentiable in f:
    f * H_m^T(g / (H_m f + s)) / sens_m (f where sens_m = 0)."""
    ghat = project(f, plan, mu, idx)
    if s_add is not None:
        ghat = ghat + s_add
    q = _safe_div(g, ghat)
    b = back_project(q, plan, mu, idx)
    pos = sens_m > 0
    return torch.where(pos, f * b / torch.where(pos, sens_m, torch.ones_like(sens_m)), f)


def subset_sensitivities(plan: Plan, n_subsets: int, mu: Optional[torch.Tensor] = None,
                         batch: Optional[int] = None) -> List[torch.Tensor]:
    """H_m^T 1 for every subset m; with a batch of attenuation maps, a (B, N, N, Nz)
    tensor per subset."""
    out = []
    for m in range(n_subsets):
        idx = subset_angles(plan.n_angles, n_subsets, m)
        if mu is not None and mu.dim() == 4:
            out.append(torch.stack([plan.sensitivity(mb, idx) for mb in mu.unbind(0)]))
        else:
            sm = plan.sensitivity(mu, idx)
            out.append(sm if batch is None else sm.expand((batch,) + sm.shape))
    return out


def unrolled_osem(plan: Plan, g: torch.Tensor, f0: torch.Tensor, n_steps: int, n_subsets: int,
                  mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                  sens: Optional[List[torch.Tensor]] = None, checkpointing: bool = True) -> torch.Tensor:
    """f_K after K = n_steps subiterations from f0 (subset k mod M), differentiable in
    f0.  With checkpointing each subiteration keeps only its input image and is
    recomputed during the backward pass."""
    batch = f0.shape[0] if f0.dim() == 4 else None
    if sens is None:
        sens = subset_sensitivities(plan, n_subsets, mu, batch)
    f = f0
    for k in range(n_steps):
        m = k % n_subsets
        idx = subset_angles(plan.n_angles, n_subsets, m)
        if checkpointing:
            f = checkpoint(osem_update, f, g, sens[m], plan, idx, mu, s_add, use_reentrant=False)
        else:
            f = osem_update(f, g, sens[m], plan, idx, mu, s_add)
    return f
