"""REINFORCE (score-function) oracle for stochastic linking -- TEST INFRASTRUCTURE ONLY.

Paper Sec. 3.2: every candidate edge between nearby particles is a Bernoulli variable and
the gradient of an expected loss is estimated by (1/S) sum_s (L_s - baseline) grad log p(y_s).

Readings fixed here (the paper is silent or uses other symbols):
  * edge probability p_e = sigmoid(z_e), z_e = (b - d_e) / tau, d_e the minimum-image
    distance (the paper's own form sigmoid(alpha (b^2 - d^2) / b^2) agrees near d = b with
    alpha = b / (2 tau));
  * the paper's own form is available too: z_e = (alpha (b^2 - d_e^2)) / b^2, evaluated in
    that order (edge_prob_quadratic), with dz_e/dx_i = -2 alpha (x_i - x_j) / b^2;
  * candidate edges: unordered pairs with d < r_c = b + 10 tau (p >= sigmoid(-10));
  * samples: y_{e,s} = [u(seed, s, i, j) < p_e] with u from Philox4x64-10 keyed by the
    seed, counter (i | j << 32, s, 0, 0) on original indices i < j;
  * grad log p(y) w.r.t. z_e is (y_e - p_e); dz_e/dx_i = -(x_i - x_j)/(tau d_e) (minimum
    image), dz_e/dx_j = +(x_i - x_j)/(tau d_e);
  * baseline: leave-one-out mean of the other samples' losses (exactly unbiased); the plain
    batch mean is available as baseline="mean".

The exhaustive enumeration over all 2^m edge subsets gives the exact gradient of E[L] for
small graphs (m <= 12); tests pin it with central finite differences of E[L].
"""
from __future__ import annotations

import ctypes
import itertools

import numpy as np

from . import _L, _pos, _ptr, OracleError, lib


def _setup():
    L = lib()
    if getattr(L, "_rf_ready", False):
        return L
    P, i64, i32, dbl, u64, u32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32)
    L.oracle_philox4x64.argtypes = [P, P, P]
    L.oracle_philox4x64.restype = None
    L.oracle_uniform.argtypes = [u64, u32, u32, u32]
    L.oracle_uniform.restype = dbl
    L.oracle_candidate_edges.argtypes = [i64, P, P, dbl, i64, P, P, P]
    L.oracle_candidate_edges.restype = i64
    L.oracle_edge_prob.argtypes = [dbl, dbl, dbl]
    L.oracle_edge_prob.restype = dbl
    L.oracle_sample_labels.argtypes = [i64, i64, P, P, P, u64, i32, P, P]
    L.oracle_sample_labels.restype = ctypes.c_int
    L._rf_ready = True
    return L


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _setup().oracle_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, s, i, j):
    return _setup().oracle_uniform(int(seed), int(s), int(i), int(j))


def candidate_edges(pos, L, r):
    """(ei, ej, d2): unordered pairs with minimum-image d^2 < r^2, ascending (i, j)."""
    pos = _pos(pos)
    n = pos.shape[0]
    cap = 1 << 16
    while True:
        ei = np.empty(cap, np.int32)
        ej = np.empty(cap, np.int32)
        d2 = np.empty(cap, np.float64)
        m = _setup().oracle_candidate_edges(n, _ptr(pos), _ptr(_L(L)), float(r), cap, _ptr(ei),
                                            _ptr(ej), _ptr(d2))
        if m < 0:
            raise OracleError(f"oracle_candidate_edges failed ({m})")
        if m <= cap:
            return ei[:m].copy(), ej[:m].copy(), d2[:m].copy()
        cap = int(m)


def edge_prob(d2, b, tau):
    L = _setup()
    return np.array([L.oracle_edge_prob(float(v), float(b), float(tau)) for v in np.asarray(d2)])


def edge_prob_quadratic(d2, b, alpha):
    """The paper's Bernoulli form (Sec. 3.2): p = sigmoid(alpha (b^2 - d^2) / b^2), FP64."""
    d2 = np.asarray(d2, np.float64)
    b2 = float(b) * float(b)
    z = (float(alpha) * (b2 - d2)) / b2
    return 1.0 / (1.0 + np.exp(-z))


def dz_factor(d, b, tau=None, alpha=None):
    """c_e with dz_e/dx_j = c_e (x_i - x_j) = -dz_e/dx_i: 1/(tau d_e) (0 when d_e = 0), or
    2 alpha / b^2 for the quadratic form."""
    d = np.asarray(d, np.float64)
    if alpha is None:
        # The distance is not differentiable where two particles coincide (d = 0); there
        # the direction (x_i - x_j)/d is undefined and the edge contributes no gradient
        # (the symmetric subgradient).
        out = np.zeros(d.shape)
        nz = d > 0.0
        out[nz] = 1.0 / (tau * d[nz])
        return out
    return np.full(d.shape, 2.0 * float(alpha) / (float(b) * float(b)))


def sample_labels(n, ei, ej, p, seed, K):
    """root[K, n] (smallest index per component of each sampled graph) and keep[K, m]."""
    ei = np.ascontiguousarray(ei, np.int32)
    ej = np.ascontiguousarray(ej, np.int32)
    p = np.ascontiguousarray(p, np.float64)
    root = np.empty((K, n), np.int32)
    keep = np.empty((K, ei.shape[0]), np.uint8)
    rc = _setup().oracle_sample_labels(n, ei.shape[0], _ptr(ei), _ptr(ej), _ptr(p), int(seed),
                                       int(K), _ptr(root), _ptr(keep))
    if rc:
        raise OracleError(f"oracle_sample_labels failed ({rc})")
    return root, keep


def edge_geometry(pos, L, ei, ej):
    """Minimum-image difference x_i - x_j (float64 [m, 3]) and distance d (float64 [m])."""
    x = pos.astype(np.float64)
    L = np.broadcast_to(np.asarray(L, np.float64), (3,))
    delta = x[ei] - x[ej]
    for a in range(3):
        da = delta[:, a]
        da[da > 0.5 * L[a]] -= L[a]
        da[da < -0.5 * L[a]] += L[a]
    d2 = delta[:, 0] * delta[:, 0] + delta[:, 1] * delta[:, 1]
    d2 = d2 + delta[:, 2] * delta[:, 2]
    return delta, np.sqrt(d2)


def score_gradient(n, ei, ej, delta, d, p, tau, keep, losses, baseline="loo", c=None):
    """(1/K) sum_s (L_s - beta_s) sum_e (y_es - p_e) dz_e/dx  ->  float64 [n, 3]; c is the
    per-edge dz factor (dz_factor), by default that of the distance form with tau."""
    K = keep.shape[0]
    Ls = np.asarray(losses, np.float64)
    if baseline == "loo":
        beta = (Ls.sum() - Ls) / max(K - 1, 1) if K > 1 else np.zeros(K)
    elif baseline == "mean":
        beta = np.full(K, Ls.mean())
    elif baseline == "none":
        beta = np.zeros(K)
    else:
        raise ValueError(baseline)
    adv = Ls - beta
    w = (adv[:, None] * (keep.astype(np.float64) - p[None, :])).sum(axis=0) / K   # [m]
    if c is None:
        c = dz_factor(d, None, tau=tau)
    dz = delta * np.asarray(c, np.float64)[:, None]                             # dz/dx_j
    g = np.zeros((n, 3))
    np.add.at(g, ei, -w[:, None] * dz)
    np.add.at(g, ej, w[:, None] * dz)
    return g


def labels_from_edges(n, ei, ej, y):
    """Smallest-index labels of the graph with the kept edges (plain union-find)."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for e in np.nonzero(y)[0]:
        ra, rb = find(int(ei[e])), find(int(ej[e]))
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(a) for a in range(n)], np.int32)


def enumerate_expectation(n, ei, ej, p, loss_fn):
    """E[L] = sum_y P(y) L(y) over all 2^m edge subsets, and the exact gradient weights
    g_e = sum_y P(y) L(y) (y_e - p_e) = d E[L] / d z_e."""
    m = ei.shape[0]
    if m > 12:
        raise ValueError("enumeration limited to 12 edges")
    EL = 0.0
    gz = np.zeros(m)
    for bits in itertools.product((0, 1), repeat=m):
        y = np.array(bits, np.uint8)
        P = float(np.prod(np.where(y == 1, p, 1.0 - p)))
        Lv = float(loss_fn(labels_from_edges(n, ei, ej, y)))
        EL += P * Lv
        gz += P * Lv * (y - p)
    return EL, gz


def _probs(d2, b, tau, alpha):
    return edge_prob(d2, b, tau) if alpha is None else edge_prob_quadratic(d2, b, alpha)


def enumerate_gradient(pos, L, b, tau, r_c, loss_fn, alpha=None):
    """Exact d E[L] / d x (float64 [n, 3]) on a small configuration by enumeration (the
    quadratic form when alpha is given)."""
    pos = _pos(pos)
    n = pos.shape[0]
    ei, ej, d2 = candidate_edges(pos, L, r_c)
    delta, d = edge_geometry(pos, L, ei, ej)
    p = _probs(d2, b, tau, alpha)
    EL, gz = enumerate_expectation(n, ei, ej, p, loss_fn)
    dz = delta * dz_factor(d, b, tau=tau, alpha=alpha)[:, None]
    g = np.zeros((n, 3))
    np.add.at(g, ei, -gz[:, None] * dz)
    np.add.at(g, ej, gz[:, None] * dz)
    return EL, g


def expected_loss(pos, L, b, tau, r_c, loss_fn, alpha=None):
    pos = _pos(pos)
    ei, ej, d2 = candidate_edges(pos, L, r_c)
    p = _probs(d2, b, tau, alpha)
    return enumerate_expectation(pos.shape[0], ei, ej, p, loss_fn)[0]


def group_sizes(root, min_size):
    """Sizes of the components with at least min_size members, in ascending label order."""
    lab, cnt = np.unique(root, return_counts=True)
    return cnt[cnt >= min_size]


def loss_sum_sq(root, min_size=2):
    """Benchmark loss: sum over kept groups of the squared member count."""
    s = group_sizes(root, min_size).astype(np.float64)
    return float((s * s).sum())
