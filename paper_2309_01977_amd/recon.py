"""OSEM reconstruction driver over the C ABI.

Section 2.1.3, Eq. 5 with the Table 1 OSEM preconditioner: the data are split
into M interleaved angle subsets; one iteration visits every subset once and
each visit is one osem_subset_step.  All state stays on the device and the
loop issues only kernel launches on the current stream (no host sync).
"""
from __future__ import annotations

from typing import List, Optional

import torch

from ._binding import Plan, subset_angles


def sensitivities(plan: Plan, n_subsets: int, mu: Optional[torch.Tensor] = None) -> List[torch.Tensor]:
    """sens_m = H_m^T 1 for every subset m (Table 1 denominator)."""
    return [plan.sensitivity(mu, subset_angles(plan.n_angles, n_subsets, m))
            for m in range(n_subsets)]


def osem(plan: Plan, g: torch.Tensor, n_iters: int, n_subsets: int,
         mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
         f0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """OSEM from f0 (default: 1 everywhere) for n_iters x n_subsets
    subiterations, as one library call (osem_reconstruct, or
    osem_reconstruct_ones without f0: the library writes the start image)."""
    if out is None:
        out = torch.empty(plan.object_shape, dtype=torch.float32, device=g.device)
    if f0 is None:
        return plan.reconstruct(g, n_iters, n_subsets, mu, s_add, f=out, from_ones=True)
    out.copy_(f0)
    return plan.reconstruct(g, n_iters, n_subsets, mu, s_add, f=out)


def osem_steps(plan: Plan, g: torch.Tensor, n_iters: int, n_subsets: int,
               mu: Optional[torch.Tensor] = None, s_add: Optional[torch.Tensor] = None,
               f0: Optional[torch.Tensor] = None, sens: Optional[List[torch.Tensor]] = None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The same reconstruction driven one subiteration at a time from Python
    (spect_sensitivity + osem_subset_step)."""
    if sens is None:
        sens = sensitivities(plan, n_subsets, mu)
    if out is None:
        out = torch.empty(plan.object_shape, dtype=torch.float32, device=g.device)
    if f0 is None:
        out.fill_(1.0)
    else:
        out.copy_(f0)
    for _ in range(n_iters):
        for m in range(n_subsets):
            plan.osem_subset_step(out, g, sens[m], m, n_subsets, mu, s_add)
    return out
