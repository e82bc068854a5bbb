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
image.  A subiteration is one library call (osem_list_step: the ratio and
the update are fused into the projector kernels) and its gradient another
(osem_list_step_vjp), which recomputes the projections from the saved input
image; no arithmetic of the update runs in PyTorch.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

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


class _Subset:
    """What one subiteration needs besides the image, as the library calls
    take it: the angle list, the measured data and additive term (full
    projection arrays; the calls read the listed rows) and sens = H_S^T 1."""

    def __init__(self, g, sens_m, idx, s_add):
        self.idx = list(idx)
        self.g, self.s, self.sens = g, s_add, sens_m


class _OsemStep(torch.autograd.Function):
    """One OSEM subiteration f * H_S^T(g / (H_S f + s)) / sens (Eq. 5 with the
    Table 1 preconditioner; osem_list_step), differentiable in f.  The
    backward is osem_list_step_vjp: it recomputes the subset's projections
    from the saved input image, so each subiteration keeps only that image
    (the recomputation that checkpointing would otherwise arrange)."""

    @staticmethod
    def forward(ctx, f, plan: Plan, sub: _Subset, mu, table):
        batched = f.dim() == 4
        f = f.contiguous()
        out = torch.empty_like(f)
        for b in range(f.shape[0] if batched else 1):
            plan.osem_list_step(f[b] if batched else f, _member(sub.g, b, batched, 3),
                                _member(sub.sens, b, batched, 3), sub.idx, _member(mu, b, batched, 3),
                                _member(table, b, batched, 1), _member(sub.s, b, batched, 3),
                                out=out[b] if batched else out)
        ctx.save_for_backward(f)
        ctx.args = (plan, sub, mu, table)
        return out

    @staticmethod
    def backward(ctx, gy):
        (f,) = ctx.saved_tensors
        plan, sub, mu, table = ctx.args
        batched = f.dim() == 4
        gy = gy.contiguous()
        gf = torch.empty_like(f)
        for b in range(f.shape[0] if batched else 1):
            plan.osem_list_step_vjp(f[b] if batched else f, _member(sub.g, b, batched, 3),
                                    _member(sub.sens, b, batched, 3), sub.idx, gy[b] if batched else gy,
                                    _member(mu, b, batched, 3), _member(table, b, batched, 1),
                                    _member(sub.s, b, batched, 3), out=gf[b] if batched else gf)
        return gf, None, None, None, None


def osem_update(f: torch.Tensor, g: torch.Tensor, sens_m: torch.Tensor, plan: Plan, idx,
                mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
                table: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One OSEM subiteration on the angles idx, differentiable in f:
    f * H_m^T(g / (H_m f + s)) / sens_m (f where sens_m = 0; the ratio 0 where
    H_m f + s <= 0).  The update and its gradient run in the library's
    kernels (osem_list_step, osem_list_step_vjp)."""
    # a table replaces the attenuation map (the library call takes one of the two)
    return _OsemStep.apply(f, plan, _Subset(g, sens_m, idx, s_add), None if table is not None else mu, table)


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
    f0.  Every subiteration keeps only its input image and recomputes its
    projections in the backward pass (osem_list_step_vjp), which is what
    checkpointing asks for; ``checkpointing`` is accepted for compatibility
    and changes nothing.  ``sens`` / ``tables`` as returned by
    subset_sensitivities (tables optional: with them every projection reads
    the attenuation factors instead of resampling mu)."""
    del checkpointing
    batch = f0.shape[0] if f0.dim() == 4 else None
    if sens is None:
        sens = subset_sensitivities(plan, n_subsets, mu, batch)
    subs = [_Subset(g, sens[m], subset_angles(plan.n_angles, n_subsets, m), s_add)
            for m in range(min(n_subsets, n_steps))]
    f = f0
    for k in range(n_steps):
        m = k % n_subsets
        # with a table the attenuation map is not passed (the call takes one or the other)
        tab = None if tables is None else tables[m]
        f = _OsemStep.apply(f, plan, subs[m], None if tab is not None else mu, tab)
    return f
