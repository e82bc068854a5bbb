"""The projector pair as torch.autograd Functions, and unrolled OSEM.

The paper builds its projectors from PyTorch operations so that they can sit
inside learned reconstruction (Section 1; the PET example of Section 3.2 hands
a PyTorch network to its deep-image-prior algorithm).  Here the system matrix H (Section 2.1.1, Eq. 1) is the HIP
forward projection and its gradient is the hand-written exact adjoint H^T
(spect_back), and vice versa; nothing is differentiated through the kernels
by autograd itself.

    project(f, plan, mu, idx)       rows idx of H f        backward: H^T
    back_project(p, plan, mu, idx)  sum_n in idx H_n^T p   backward: H (rows idx)

Both may read the attenuation factors from a table written once per angle
list (Plan.sensitivity_table) instead of forming them from mu each time.

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


def _member(a: Optional[torch.Tensor], b: int, batched: bool, rank: int):
    """Member b's attenuation map (rank 3) or table (rank 1) of a batch, or
    the one shared by the batch."""
    if a is None:
        return None
    if batched and a.dim() == rank + 1:
        return a[b]
    return a


def _fwd(plan: Plan, x, mu, table, idx):
    return plan.forward(x, mu, idx) if table is None else plan.forward_table(x, table, idx)


def _back(plan: Plan, y, mu, table, idx):
    return plan.back(y, mu, idx) if table is None else plan.back_table(y, table, idx)


class _Pair(torch.autograd.Function):
    """H (adjoint=False) or H^T (adjoint=True); the backward applies the other."""

    @staticmethod
    def forward(ctx, x, plan: Plan, mu, table, idx, adjoint: bool):
        ctx.plan, ctx.idx, ctx.adjoint = plan, idx, adjoint
        ctx.mu, ctx.table = mu, table
        batched = x.dim() == 4
        op = _back if adjoint else _fwd
        outs = [op(plan, xb, _member(mu, b, batched, 3), _member(table, b, batched, 1), idx)
                for b, xb in enumerate(_members(x.contiguous(), 3))]
        return torch.stack(outs) if batched else outs[0]

    @staticmethod
    def backward(ctx, gy):
        batched = gy.dim() == 4
        op = _fwd if ctx.adjoint else _back
        outs = [op(ctx.plan, gb, _member(ctx.mu, b, batched, 3), _member(ctx.table, b, batched, 1), ctx.idx)
                for b, gb in enumerate(_members(gy.contiguous(), 3))]
        return (torch.stack(outs) if batched else outs[0]), None, None, None, None, None


def project(f: torch.Tensor, plan: Plan, mu: Optional[torch.Tensor] = None,
            idx: Optional[Sequence[int]] = None, table: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Rows idx of H f (zeros elsewhere); differentiable in f.  With ``table``
    (from Plan.sensitivity_table for the same idx; (B, T) for a batch) the
    attenuation factors are read from it instead of being formed from mu."""
    return _Pair.apply(f, plan, mu, table, None if idx is None else list(idx), False)


def back_project(p: torch.Tensor, plan: Plan, mu: Optional[torch.Tensor] = None,
                 idx: Optional[Sequence[int]] = None, table: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum over n in idx of H_n^T p[n]; differentiable in p (``table`` as in project)."""
    return _Pair.apply(p, plan, mu, table, None if idx is None else list(idx), True)


def _safe_div(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """a / b where b > 0, else 0 (the 0/0 reading of the ratio)."""
    pos = b > 0
    return torch.where(pos, a / torch.where(pos, b, torch.ones_like(b)), torch.zeros_like(a))


def osem_update(f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, plan: Plan, idx,
                mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                table: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One OSEM subiteration on the angles idx, differentiable in f:
    f * H_m^T(g / (H_m f + s)) / sens_m (f where sens_m = 0)."""
    ghat = project(f, plan, mu, idx, table)
    if s_add is not None:
        ghat = ghat + s_add
    q = _safe_div(g, ghat)
    b = back_project(q, plan, mu, idx, table)
    pos = sens_m > 0
    return torch.where(pos, f * b / torch.where(pos, sens_m, torch.ones_like(sens_m)), f)


def subset_sensitivities(plan: Plan, n_subsets: int, mu: Optional[torch.Tensor] = None,
                         batch: Optional[int] = None, tables: bool = False):
    """H_m^T 1 for every subset m (a (B, N, N, Nz) tensor per subset for a
    batch of attenuation maps).  With tables=True (mu required) returns
    (sensitivities, tables): the attenuation-factor table of every subset,
    (B, T) per subset for a batch, written by the same pass."""
    if tables and mu is None:
        raise ValueError("attenuation tables need an attenuation map")
    batched_mu = mu is not None and mu.dim() == 4
    maps = list(mu.unbind(0)) if batched_mu else [mu]
    sens, tabs = [], []
    for m in range(n_subsets):
        idx = subset_angles(plan.n_angles, n_subsets, m)
        if tables:
            tb = torch.empty((len(maps), plan.table_size(len(idx)) // 4), dtype=torch.float32, device="cuda")
            sm = [plan.sensitivity_table(mb, idx, table=tb[b])[0] for b, mb in enumerate(maps)]
            tabs.append(tb if batched_mu else tb[0])
        else:
            sm = [plan.sensitivity(mb, idx) for mb in maps]
        if batched_mu:
            sens.append(torch.stack(sm))
        else:
            sens.append(sm[0] if batch is None else sm[0].expand((batch,) + sm[0].shape))
    return (sens, tabs) if tables else sens


def unrolled_osem(plan: Plan, g: torch.Tensor, f0: torch.Tensor, n_steps: int, n_subsets: int,
                  mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                  sens: Optional[List[torch.Tensor]] = None, tables: Optional[List[torch.Tensor]] = None,
                  checkpointing: bool = True) -> torch.Tensor:
    """f_K after K = n_steps subiterations from f0 (subset k mod M), differentiable in
    f0.  With checkpointing each subiteration keeps only its input image and is
    recomputed during the backward pass.  ``sens`` / ``tables`` as returned by
    subset_sensitivities (tables optional: with them every projection reads
    the attenuation factors instead of resampling mu)."""
    batch = f0.shape[0] if f0.dim() == 4 else None
    if sens is None:
        sens = subset_sensitivities(plan, n_subsets, mu, batch)
    f = f0
    for k in range(n_steps):
        m = k % n_subsets
        idx = subset_angles(plan.n_angles, n_subsets, m)
        tab = None if tables is None else tables[m]
        if checkpointing:
            f = checkpoint(osem_update, f, g, sens[m], plan, idx, mu, s_add, tab, use_reentrant=False)
        else:
            f = osem_update(f, g, sens[m], plan, idx, mu, s_add, tab)
    return f
