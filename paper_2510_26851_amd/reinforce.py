"""Stochastic linking and the REINFORCE gradient (paper Sec. 3.2) through libfof.so.

    smp = Sampler(pos, L, b, tau, K, seed)     # cut radius r_c = b + 10 tau by default
    smp.sample()                               # K sampled graphs, linked on the GPU
    halos = smp.groups(min_size=2)             # per-sample sizes and centres (device tables)
    losses = sum_sq_sizes(halos)               # any function of the tables (float64 [K])
    grad = smp.grad(losses, baseline="loo")    # float32 [n, 3]: score-function estimate

Edge e = {i, j} (pairs closer than r_c) is kept in sample s with probability
sigmoid((b - d_e) / tau), decided by the Philox4x64-10 uniform documented in include/fof.h.
Every step of the method (candidate edges, sampling, components, group sizes and centres, the
estimator) runs in the library; the loss is the caller's function of the group tables.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check
from .fof import Plan, _need, _ptr, _stream

_BASELINES = {"none": _lib.FOF_BASELINE_NONE, "mean": _lib.FOF_BASELINE_MEAN,
              "loo": _lib.FOF_BASELINE_LOO}


class Sampler:
    """Without an explicit edge_cap the capacity fits itself on the first sample(): it reads
    the edge count back (one synchronisation) and, if it exceeded the capacity or left most
    of it unused, reallocates and runs again (the per-sample passes scale with the
    capacity).  With an explicit edge_cap an overflow only sets FOF_STATUS_EDGE_CAP.

    Samples s_first .. s_first + K - 1 are drawn, so K samplers of one sample each with
    s_first = 0 .. K - 1 draw exactly the graphs of one sampler of K."""

    def __init__(self, pos, L, b, tau, K, seed, r_cut=None, edge_cap=None, tune=None,
                 alpha=None, s_first=0):
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
        self.s_first = int(s_first)
        self.b, self.tau, self.seed = float(b), float(tau), int(seed)
        self.auto_fit = edge_cap is None
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
        S.form, S.alpha, S.s_first = self.form, self.alpha, self.s_first
        self.S = S
        self.vcap = min(2 * cap, self.n)

    def _launch(self, root, stream):
        check("fof_link", _lib.load().fof_link(self.plan._gref, _ptr(self.plan.ws),
                                               self.plan.ws_bytes, ctypes.byref(self.S),
                                               _ptr(root), _stream(stream)))

    def sample(self, root=None, want_labels=False, stream=None):
        """Draws and links the K graphs.  With want_labels (or a root tensor given) also
        returns their labels, int32 [K, n] (the smallest member index per component)."""
        want_labels = want_labels or root is not None
        if want_labels and root is None:
            root = torch.empty((self.K, self.n), dtype=torch.int32, device=self.device)
        self._launch(root, stream)
        if self.auto_fit:
            self.auto_fit = False
            total = int(self.n_edges.item())
            cap = self.S.edge_cap
            if total > cap or cap > 2 * total + 65536:
                self._alloc(total + total // 8 + 1024)
                self.plan.build_grid(self.pos, stream)  # clears the overflow status bit
                self._launch(root, stream)
        return root

    def groups(self, min_size=2, cap=None, out=None, stream=None):
        """Halos of every sampled graph of the last sample(): components with at least
        min_size (>= 2) members, in ascending label order.  Returns device tensors
        n_groups int32 [K], sizes int32 [K, cap], com float64 [K, cap, 3] (entries past
        n_groups[k] are unspecified) and cap.  The default cap, vcap // 2, cannot overflow.
        Tensors passed in `out` (a previous result) are reused; they must have the shapes of
        this cap (by default the cap they were made for), else ValueError."""
        o = out or {}
        if cap is None:
            cap = int(o["cap"]) if "cap" in o else max(1, self.vcap // 2)
        cap = int(cap)
        d, K = self.device, self.K

        def buf(name, dtype, shape):
            t = o.get(name)
            if t is None:
                return torch.empty(shape, dtype=dtype, device=d)
            _need(t, name, dtype, shape, d)
            return t

        ng = buf("n_groups", torch.int32, (K,))
        sizes = buf("sizes", torch.int32, (K, cap))
        com = buf("com", torch.float64, (K, cap, 3))
        check("fof_groups",
              _lib.load().fof_groups(self.plan._gref, _ptr(self.plan.ws), self.plan.ws_bytes,
                                     ctypes.byref(self.S), int(min_size), None, cap, None,
                                     _ptr(ng), _ptr(sizes), _ptr(com), None, None,
                                     _stream(stream)))
        return dict(n_groups=ng, sizes=sizes, com=com, cap=cap)

    def edges(self):
        m = min(int(self.n_edges.item()), self.S.edge_cap)
        return self.ei[:m], self.ej[:m], self.d2[:m], int(self.n_edges.item())

    def grad(self, losses, baseline="loo", stream=None, out=None):
        loss = losses.to(device=self.device, dtype=torch.float64).contiguous()
        assert loss.shape == (self.K,)
        gp = out if out is not None else torch.empty((self.n, 3), dtype=torch.float32,
                                                     device=self.device)
        check("fof_backward",
              _lib.load().fof_backward(self.plan._gref, _ptr(self.plan.ws), self.plan.ws_bytes,
                                       _lib.FOF_SCORE, None, 0, None, None, None, None, None,
                                       None, None, ctypes.byref(self.S), _ptr(loss),
                                       _BASELINES[baseline], _ptr(gp), None, _stream(stream)))
        return gp


def valid(halos):
    """bool [K, cap]: which table entries hold a group."""
    cap = halos["cap"]
    g = torch.arange(cap, device=halos["sizes"].device).reshape(1, cap)
    return g < halos["n_groups"].reshape(-1, 1)


def sum_sq_sizes(halos):
    """Per-sample loss sum_g n_g^2 over the groups of the tables (float64 [K])."""
    n = halos["sizes"].to(torch.float64)
    return torch.where(valid(halos), n * n, torch.zeros_like(n)).sum(dim=1)
