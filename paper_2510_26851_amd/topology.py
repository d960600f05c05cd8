"""Toy topology optimisation with the REINFORCE estimator (paper Sec. 3.2, toy problem).

Particles move so that halos (components of at least `min_mass` members of a sampled link
graph) form inside a target region Omega and break up outside it.  The loss of one sampled
graph is the paper's
    L = sum_{H not in Omega} M_H - sum_{H in Omega} M_H,
M_H the member count, a halo being in Omega when its centre (members unwrapped about the
label particle by minimum image, averaged, wrapped into the box) is.  Each step samples K
graphs with the stochastic linking of the library (edge probability sigmoid of
alpha (b^2 - d^2) / b^2), scores them, and applies the estimated gradient with Adam.  The
sampling and the score gradient run in the HIP kernels; the loss, a function of K label
arrays, is plain PyTorch.
"""
from __future__ import annotations

import torch

from .reinforce import Sampler


def halo_mass_loss(pos, root, L, min_mass, inside):
    """Per-sample loss (float64 [K]) for labels root (int [K, n], smallest member index) of
    particles pos (float32 [n, 3]) in a periodic box L; inside(com [H, 3]) -> bool [H]."""
    K, n = root.shape
    dev = pos.device
    Lt = torch.as_tensor(L, dtype=torch.float64, device=dev).reshape(1, -1).expand(1, 3)
    x = pos.to(torch.float64)
    lab = root.long()
    flat = (lab + n * torch.arange(K, device=dev).reshape(K, 1)).reshape(-1)   # [K n]
    count = torch.bincount(flat, minlength=K * n)
    d = x.repeat(K, 1) - x[lab.reshape(-1)]
    d = torch.where(d > Lt / 2, d - Lt, torch.where(d < -Lt / 2, d + Lt, d))
    s = torch.zeros((K * n, 3), dtype=torch.float64, device=dev).index_add_(0, flat, d)
    halo = torch.nonzero(count >= min_mass).reshape(-1)                        # label slots
    mass = count[halo].to(torch.float64)
    com = torch.remainder(x[halo % n] + s[halo] / mass.reshape(-1, 1), Lt)
    sign = torch.where(inside(com), -1.0, 1.0).to(torch.float64)
    return torch.zeros(K, dtype=torch.float64, device=dev).index_add_(0, halo // n, sign * mass)


def optimise(pos, L, b, alpha, K, steps, lr, min_mass, inside, seed=0, baseline="mean"):
    """Adam on the particle positions for `steps` iterations (positions stay wrapped in the
    box); returns the final positions and the mean sampled loss of every step."""
    p = torch.nn.Parameter(pos.detach().clone())
    opt = torch.optim.Adam([p], lr=lr)
    Lt = torch.as_tensor(L, dtype=torch.float32, device=pos.device)
    history = []
    for it in range(steps):
        smp = Sampler(p.detach(), L, b, None, K, seed + it, alpha=alpha)
        root = smp.sample()
        losses = halo_mass_loss(p.detach(), root, L, min_mass, inside)
        p.grad = smp.grad(losses, baseline=baseline)
        opt.step()
        with torch.no_grad():
            p.copy_(torch.remainder(p, Lt))
            p.masked_fill_(p >= Lt, 0.0)  # remainder can round up to L in float32
        history.append(float(losses.mean()))
    return p.detach(), history
