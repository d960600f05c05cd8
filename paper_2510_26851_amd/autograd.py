"""Differentiable group statistics with frozen assignment (paper Sec. 3.1).

The forward runs the exact Friends-of-Friends pass (binning, linking, groups) in the HIP
library; the backward holds memberships fixed and calls fof_backward:
    d com_g / d x_i = 1 / n_g,   d mass_g / d (x, v) = 0,
    d sigv_g / d v_ic = (v_ic - vmean_gc) / (3 n_g sigv_g).
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
