"""Stochastic linking and the REINFORCE gradient (paper Sec. 3.2) through libfof.so.

    smp = Sampler(pos, L, b, tau, K, seed)     # cut radius r_c = b + 10 tau by default
    root = smp.sample()                        # int32 [K, n]: labels of the K sampled graphs
    grad = smp.grad(losses, baseline="loo")    # float32 [n, 3]: score-function estimate

Edge e = {i, j} (pairs closer than r_c) is kept in sample s with probability
sigmoid((b - d_e) / tau), decided by the Philox4x64-10 uniform documented in include/fof.h.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check
from .fof import Plan, _ptr, _stream

_BASELINES = {"none": _lib.FOF_BASELINE_NONE, "mean": _lib.FOF_BASELINE_MEAN,
              "loo": _lib.FOF_BASELINE_LOO}


class Sampler:
    """Without an explicit edge_cap the capacity grows on demand: sample() reads the edge
    count back (one synchronisation) and, if it exceeded the capacity, reallocates and runs
    again.  With an explicit edge_cap an overflow only sets FOF_STATUS_EDGE_CAP."""

    def __init__(self, pos, L, b, tau, K, seed, r_cut=None, edge_cap=None, tune=None,
                 alpha=None):
        # alpha given: the paper's form z = alpha (b^2 - d^2) / b^2 (tau unused); otherwise
        # z = (b - d) / tau.  Default cut: the distance where z = -10 (p = sigmoid(-10)).
        self.n = pos.shape[0]
        self.device = pos.device
        self.form = _lib.FOF_PROB_DISTANCE if alpha is None else _lib.FOF_PROB_QUADRATIC
        self.alpha = 0.0 if alpha is None else float(alpha)
        if tau is None:
            tau = 0.0
        if r_cut is None:
            r_cut = (b + 10.0 * tau if alpha is None
                     else b * (1.0 + 10.0 / float(alpha)) ** 0.5)
        self.r_cut = float(r_cut)
        self.plan = Plan([self.n], [(L, self.r_cut)], device=pos.device, tune=tune)
        self.pos = pos
        self.K = int(K)
        self.b, self.tau, self.seed = float(b), float(tau), int(seed)
        self.auto_grow = edge_cap is None
        self._alloc(int(edge_cap) if edge_cap is not None else max(1024, 4 * self.n))
        self.plan.build_grid(pos)

    def _alloc(self, cap):
        d = self.device
        self.ei = torch.empty(cap, dtype=torch.int32, device=d)
        self.ej = torch.empty(cap, dtype=torch.int32, device=d)
        self.d2 = torch.empty(cap, dtype=torch.float64, device=d)
        self.n_edges = torch.zeros(1, dtype=torch.int32, device=d)
        nb = _lib.sample_scratch_bytes(self.n, self.K, cap)
        self.scratch = torch.empty(nb, dtype=torch.uint8, device=d)
        S = _lib.fof_sample()
        S.b, S.tau, S.seed, S.K, S.edge_cap = self.b, self.tau, self.seed, self.K, cap
        S.ei, S.ej, S.d2 = self.ei.data_ptr(), self.ej.data_ptr(), self.d2.data_ptr()
        S.n_edges = self.n_edges.data_ptr()
        S.scratch, S.scratch_bytes = self.scratch.data_ptr(), nb
        S.form, S.alpha = self.form, self.alpha
        self.S = S

    def _launch(self, root, stream):
        check("fof_link", _lib.load().fof_link(self.plan._gref, _ptr(self.plan.ws),
                                               ctypes.byref(self.S), _ptr(root), _stream(stream)))

    def sample(self, root=None, want_labels=True, stream=None):
        if want_labels and root is None:
            root = torch.empty((self.K, self.n), dtype=torch.int32, device=self.device)
        root = root if want_labels else None
        self._launch(root, stream)
        if self.auto_grow:
            total = int(self.n_edges.item())
            if total > self.S.edge_cap:
                self._alloc(total + total // 8 + 1024)
                self.plan.build_grid(self.pos, stream)  # clears the overflow status bit
                self._launch(root, stream)
        return root

    def edges(self):
        m = min(int(self.n_edges.item()), self.S.edge_cap)
        return self.ei[:m], self.ej[:m], self.d2[:m], int(self.n_edges.item())

    def grad(self, losses, baseline="loo", stream=None):
        loss = losses.to(device=self.device, dtype=torch.float64).contiguous()
        assert loss.shape == (self.K,)
        gp = torch.empty((self.n, 3), dtype=torch.float32, device=self.device)
        check("fof_backward",
              _lib.load().fof_backward(self.plan._gref, _ptr(self.plan.ws), _lib.FOF_SCORE, None,
                                       0, None, None, None, None, None, None, None,
                                       ctypes.byref(self.S), _ptr(loss), _BASELINES[baseline],
                                       _ptr(gp), None, _stream(stream)))
        return gp


def sum_sq_sizes(root, min_size=2):
    """Per-sample loss sum_g n_g^2 over groups with at least min_size members (torch)."""
    K, n = root.shape
    out = torch.empty(K, dtype=torch.float64, device=root.device)
    for s in range(K):
        c = torch.bincount(root[s].long(), minlength=n)
        c = c[c >= min_size].to(torch.float64)
        out[s] = (c * c).sum()
    return out
