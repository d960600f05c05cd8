"""Toy topology optimisation with the REINFORCE estimator (paper Sec. 3.2, toy problem).

Particles move so that halos (components of at least `min_mass` members of a sampled link
graph) form inside a target region Omega and break up outside it.  The loss of one sampled
graph is the paper's
    L = sum_{H not in Omega} M_H - sum_{H in Omega} M_H,
M_H the member count, a halo being in Omega when its centre (members unwrapped about the
label particle by minimum image, averaged, wrapped into the box) is.  Each step samples K
graphs with the stochastic linking of the library (edge probability sigmoid of
alpha (b^2 - d^2) / b^2), builds their halos (sizes and centres per sample), scores them,
and applies the estimated gradient with Adam.  Sampling, halos and the score gradient run
in the HIP kernels; the loss, a signed sum over each sample's halo table, is PyTorch.
"""
from __future__ import annotations

import torch

from .reinforce import Sampler, valid


def halo_mass_loss(halos, inside):
    """Per-sample loss (float64 [K]) from the group tables of Sampler.groups (halos of at
    least the minimum mass, their member counts and centres, built on the GPU);
    inside(com [K, cap, 3]) -> bool [K, cap] tells which centres lie in Omega."""
    mass = halos["sizes"].to(torch.float64)
    sign = torch.where(inside(halos["com"]), -1.0, 1.0).to(torch.float64)
    return torch.where(valid(halos), sign * mass, torch.zeros_like(mass)).sum(dim=1)


def optimise(pos, L, b, alpha, K, steps, lr, min_mass, inside, seed=0, baseline="mean"):
    """Adam on the particle positions for `steps` iterations (positions stay wrapped in the
    box); returns the final positions and the mean sampled loss of every step."""
    p = torch.nn.Parameter(pos.detach().clone())
    opt = torch.optim.Adam([p], lr=lr)
    Lt = torch.as_tensor(L, dtype=torch.float32, device=pos.device)
    history = []
    for it in range(steps):
        smp = Sampler(p.detach(), L, b, None, K, seed + it, alpha=alpha)
        smp.sample()
        losses = halo_mass_loss(smp.groups(min_mass), inside)
        p.grad = smp.grad(losses, baseline=baseline)
        opt.step()
        with torch.no_grad():
            p.copy_(torch.remainder(p, Lt))
            p.masked_fill_(p >= Lt, 0.0)  # remainder can round up to L in float32
        history.append(float(losses.mean()))
    return p.detach(), history
