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


def _fwd(plan: Plan, x, mu, table, idx, out):
    return plan.forward(x, mu, idx, out) if table is None else plan.forward_table(x, table, idx, out)


def _back(plan: Plan, y, mu, table, idx, out):
    return plan.back(y, mu, idx, out) if table is None else plan.back_table(y, table, idx, out)


def _apply(plan: Plan, x, mu, table, idx, adjoint: bool):
    """H x (rows idx, zeros elsewhere) or H^T x, member by member straight into
    one output tensor (no per-member results to stack)."""
    batched = x.dim() == 4
    x = x.contiguous()
    lead = (x.shape[0],) if batched else ()
    if adjoint:
        out = torch.empty(lead + plan.object_shape, dtype=torch.float32, device=x.device)
    else:
        out = torch.zeros(lead + plan.proj_shape, dtype=torch.float32, device=x.device)
    op = _back if adjoint else _fwd
    for b, xb in enumerate(_members(x, 3)):
        op(plan, xb, _member(mu, b, batched, 3), _member(table, b, batched, 1), idx, out[b] if batched else out)
    return out


class _Pair(torch.autograd.Function):
    """H (adjoint=False) or H^T (adjoint=True); the backward applies the other."""

    @staticmethod
    def forward(ctx, x, plan: Plan, mu, table, idx, adjoint: bool):
        ctx.plan, ctx.idx, ctx.adjoint = plan, idx, adjoint
        ctx.mu, ctx.table = mu, table
        return _apply(plan, x, mu, table, idx, adjoint)

    @staticmethod
    def backward(ctx, gy):
        return _apply(ctx.plan, gy, ctx.mu, ctx.table, ctx.idx, not ctx.adjoint), None, None, None, None, None


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


def _rows_apply(plan: Plan, x, mu, table, idx, rows, adjoint: bool):
    """adjoint=False: the rows idx of H x as a compact (..., len(idx), N, Nz)
    tensor; adjoint=True: H^T of such compact rows.  The full projection
    buffer the calls take is left unfilled outside the rows idx: the forward
    writes and the back projection reads no other row."""
    batched = x.dim() == 4
    x = x.contiguous()
    lead = (x.shape[0],) if batched else ()
    full = torch.empty(lead + plan.proj_shape, dtype=torch.float32, device=x.device)
    if adjoint:
        full.index_copy_(-3, rows, x)
        out = torch.empty(lead + plan.object_shape, dtype=torch.float32, device=x.device)
        for b in range(x.shape[0] if batched else 1):
            _back(plan, full[b] if batched else full, _member(mu, b, batched, 3), _member(table, b, batched, 1),
                  idx, out[b] if batched else out)
        return out
    for b, xb in enumerate(_members(x, 3)):
        _fwd(plan, xb, _member(mu, b, batched, 3), _member(table, b, batched, 1), idx,
             full[b] if batched else full)
    return full.index_select(-3, rows)


class _Rows(torch.autograd.Function):
    """Compact-row form of the pair (see _rows_apply); the backward applies
    the other operator."""

    @staticmethod
    def forward(ctx, x, plan: Plan, mu, table, idx, rows, adjoint: bool):
        ctx.args = (plan, mu, table, idx, rows, adjoint)
        return _rows_apply(plan, x, mu, table, idx, rows, adjoint)

    @staticmethod
    def backward(ctx, gy):
        plan, mu, table, idx, rows, adjoint = ctx.args
        return _rows_apply(plan, gy, mu, table, idx, rows, not adjoint), None, None, None, None, None, None


class _Subset:
    """What one subiteration needs that does not depend on the image: the
    subset's rows, the measured (and additive) rows, where sens_m > 0 and
    sens_m with 1 where it is 0."""

    def __init__(self, g, sens_m, idx, s_add, device):
        self.idx = list(idx)
        self.rows = torch.as_tensor(self.idx, dtype=torch.long, device=device)
        self.g = g.index_select(-3, self.rows)
        self.s = None if s_add is None else s_add.index_select(-3, self.rows)
        self.pos = sens_m > 0
        self.sens = torch.where(self.pos, sens_m, torch.ones_like(sens_m))


def _osem_step(f, sub: _Subset, plan: Plan, mu, table):
    gh = _Rows.apply(f, plan, mu, table, sub.idx, sub.rows, False)
    if sub.s is not None:
        gh = gh + sub.s
    b = _Rows.apply(_safe_div(sub.g, gh), plan, mu, table, sub.idx, sub.rows, True)
    return torch.where(sub.pos, f * b / sub.sens, f)


def osem_update(f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, plan: Plan, idx,
                mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                table: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One OSEM subiteration on the angles idx, differentiable in f:
    f * H_m^T(g / (H_m f + s)) / sens_m (f where sens_m = 0).  The ratio is
    formed on the rows idx only: H_m^T reads no other row."""
    return _osem_step(f, _Subset(g, sens_m, idx, s_add, f.device), plan, mu, table)


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
    subs = [_Subset(g, sens[m], subset_angles(plan.n_angles, n_subsets, m), s_add, f0.device)
            for m in range(min(n_subsets, n_steps))]
    f = f0
    for k in range(n_steps):
        m = k % n_subsets
        tab = None if tables is None else tables[m]
        if checkpointing:
            f = checkpoint(_osem_step, f, subs[m], plan, mu, tab, use_reentrant=False)
        else:
            f = _osem_step(f, subs[m], plan, mu, tab)
    return f
