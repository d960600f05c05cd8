"""Differentiable group statistics with frozen assignment (paper Sec. 3.1).

The forward runs the exact Friends-of-Friends pass (binning, linking, groups) in the HIP
library; the backward holds memberships fixed and calls fof_backward:
    d com_g / d x_i = 1 / n_g,   d mass_g / d (x, v) = 0,
    d sigv_g / d v_ic = (v_ic - vmean_gc) / (3 n_g sigv_g).

Decorated frozen assignment (Sec. 3.1): the position dispersion sigx_g of each group is a
differentiable proxy ("decoration") for its mass; its gradient is
    d sigx_g / d x_ic = mi(x_ic - com_gc) / (3 n_g sigx_g)
(fof_group_dispersion / fof_backward_dispersion).  soft_histogram lets derivatives of a
histogram of such values, e.g. a halo mass function in sigx, flow between bins.
"""
from __future__ import annotations

import torch

from .fof import Plan


class FoFStats(torch.autograd.Function):
    """(pos, vel) -> (mass[G], com[G, 3], sigv[G]) for the groups of one batch plan.

    mass is the member count (particle mass 1) in float64; com and sigv are float64.
    """

    @staticmethod
    def forward(ctx, pos, vel, plan: Plan, min_size: int):
        plan.build_grid(pos.detach())
        plan.link()
        res = plan.groups(min_size, vel=vel.detach())
        G = int(res["n_groups"].item())
        k = min(G, res["cap"])
        sizes = res["sizes"][:k]
        com = res["com"][:k]
        vmean = res["vmean"][:k]
        sigv = res["sigv"][:k]
        ctx.plan = plan
        ctx.G = k
        ctx.save_for_backward(res["group_id"], sizes, vmean, sigv, vel.detach())
        ctx.mark_non_differentiable(res["group_id"])
        return sizes.to(torch.float64), com, sigv, res["group_id"]

    @staticmethod
    def backward(ctx, g_mass, g_com, g_sigv, _g_gid):
        group_id, sizes, vmean, sigv, vel = ctx.saved_tensors
        gp, gv = ctx.plan.backward(group_id, ctx.G, sizes, vmean=vmean, sigv=sigv, vel=vel,
                                   g_mass=g_mass, g_com=g_com, g_sigv=g_sigv,
                                   want_pos=ctx.needs_input_grad[0],
                                   want_vel=ctx.needs_input_grad[1])
        return gp, gv, None, None


def fof_stats(pos, vel, L, b, min_size=20, plan=None):
    """Differentiable (mass, com, sigv, group_id) of one periodic box."""
    if plan is None:
        plan = Plan([pos.shape[0]], [(L, b)], device=pos.device)
    return FoFStats.apply(pos, vel, plan, min_size)


class FoFDecorated(torch.autograd.Function):
    """pos -> (mass[G], com[G, 3], sigx[G], group_id) for the groups of one batch plan, with
    memberships frozen; sigx is the position dispersion (float64)."""

    @staticmethod
    def forward(ctx, pos, plan: Plan, min_size: int):
        plan.build_grid(pos.detach())
        plan.link()
        res = plan.groups(min_size)
        sig = plan.dispersion(res)
        G = int(res["n_groups"].item())
        k = min(G, res["cap"])
        sizes = res["sizes"][:k]
        com = res["com"][:k]
        sigx = sig[:k]
        ctx.plan = plan
        ctx.G = k
        ctx.save_for_backward(pos.detach(), res["group_id"], sizes, com, sigx)
        ctx.mark_non_differentiable(res["group_id"])
        return sizes.to(torch.float64), com, sigx, res["group_id"]

    @staticmethod
    def backward(ctx, g_mass, g_com, g_sigx, _g_gid):
        pos, group_id, sizes, com, sigx = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None
        gp, _ = ctx.plan.backward(group_id, ctx.G, sizes, g_mass=g_mass, g_com=g_com,
                                  want_pos=True, want_vel=False)
        if g_sigx is not None:
            ctx.plan.backward_dispersion(pos, group_id, ctx.G, sizes, com, sigx, g_sigx, gp)
        return gp, None, None


def fof_decorated(pos, L, b, min_size=20, plan=None):
    """Differentiable (mass, com, sigx, group_id) of one periodic box (decorated frozen
    assignment)."""
    if plan is None:
        plan = Plan([pos.shape[0]], [(L, b)], device=pos.device)
    return FoFDecorated.apply(pos, plan, min_size)


def soft_histogram(values, edges, width):
    """Soft histogram: bin k of edges [e_k, e_{k+1}) counts
    sum_g sigmoid((v_g - e_k) / width) - sigmoid((v_g - e_{k+1}) / width),
    which tends to the ordinary count as width -> 0 and passes derivatives to every value
    near a bin edge (plain PyTorch; values is a short per-group vector)."""
    v = values.reshape(-1, 1)
    lo = edges[:-1].reshape(1, -1)
    hi = edges[1:].reshape(1, -1)
    return (torch.sigmoid((v - lo) / width) - torch.sigmoid((v - hi) / width)).sum(dim=0)

