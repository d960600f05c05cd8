"""Pins of the REINFORCE oracle (paper Sec. 3.2) against things other than itself.

* Philox4x64-10: numpy.random.Philox is an independent implementation of the same
  published generator (it advances the 256-bit counter by one before each block).
* candidate edges: all-pairs numpy distances.
* sampled labels: scipy connected components of the kept edges, and the uniform stream.
* enumeration: a single edge has E[L] = p and dE/dz = p (1 - p) in closed form; on small
  random graphs the enumerated score-function gradient equals central finite differences of
  the enumerated expectation.
* estimator: the Monte-Carlo mean of the score-function estimate converges to the exact
  gradient (z-test), with the leave-one-out baseline exactly unbiased.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import workloads as W
from oracle import reinforce as RF

MASK64 = (1 << 64) - 1


def numpy_philox_block(ctr, key):
    """Philox4x64-10 output for counter `ctr` through numpy's generator, which increments
    the counter before producing each block of four words."""
    c = sum(int(v) << (64 * k) for k, v in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    prev = [(c >> (64 * k)) & MASK64 for k in range(4)]
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [0, 0]),
    ([0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89],
     [0x452821E638D01377, 0xBE5466CF34E90C6C]),
    ([MASK64, MASK64, MASK64, MASK64], [MASK64, MASK64]),
    ([12345 | (678 << 32), 63, 0, 0], [26951, 0]),
])
def test_philox_matches_numpy(ctr, key):
    got = RF.philox4x64(ctr, key)
    ref = numpy_philox_block(ctr, key)
    np.testing.assert_array_equal(got, ref)


def test_philox_random_counters_match_numpy():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2)]
        np.testing.assert_array_equal(RF.philox4x64(ctr, key), numpy_philox_block(ctr, key))


def test_uniform_stream_definition():
    seed, s, i, j = 26951, 5, 17, 4242
    out = numpy_philox_block([i | (j << 32), s, 0, 0], [seed, 0])
    assert RF.uniform(seed, s, i, j) == float(int(out[0]) >> 11) * 2.0 ** -53
    us = np.array([RF.uniform(seed, s, i, jj) for jj in range(20000, 24000)])
    assert 0.0 <= us.min() and us.max() < 1.0
    assert abs(us.mean() - 0.5) < 0.02


def brute_edges(pos, L, r):
    x = pos.astype(np.float64)
    Lv = np.broadcast_to(np.asarray(L, np.float64), (3,))
    out = []
    for i in range(x.shape[0] - 1):
        d = x[i] - x[i + 1:]
        for a in range(3):
            da = d[:, a]
            da[da > 0.5 * Lv[a]] -= Lv[a]
            da[da < -0.5 * Lv[a]] += Lv[a]
        s = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
        s = s + d[:, 2] * d[:, 2]
        for j in np.nonzero(s < r * r)[0]:
            out.append((i, i + 1 + j, s[j]))
    return out


@pytest.mark.parametrize("seed,n,L,r", [(1, 400, 6.0, 0.6), (2, 1000, 10.0, 0.75), (3, 60, 1.0, 0.3)])
def test_candidate_edges_match_brute_force(seed, n, L, r):
    pos = W.uniform_box(n, (L, L, L), seed)
    ei, ej, d2 = RF.candidate_edges(pos, L, r)
    ref = brute_edges(pos, L, r)
    assert [(int(a), int(b)) for a, b in zip(ei, ej)] == [(a, b) for a, b, _ in ref]
    np.testing.assert_array_equal(d2, [s for _, _, s in ref])


def test_edge_probability_closed_form():
    b, tau = 0.2, 0.01
    for d in [0.0, 0.1, 0.19, 0.2, 0.21, 0.3]:
        p = RF.edge_prob(np.array([d * d]), b, tau)[0]
        z = (b - d) / tau
        assert abs(p - 1.0 / (1.0 + np.exp(-z))) <= 1e-15
    assert RF.edge_prob(np.array([0.04]), 0.2, 0.01)[0] == 0.5


def test_sampled_labels_match_components_of_kept_edges():
    pos = W.clumpy_box(600, 8.0, 3, 5)
    b, tau = 0.3, 0.015
    ei, ej, d2 = RF.candidate_edges(pos, 8.0, b + 10 * tau)
    p = RF.edge_prob(d2, b, tau)
    root, keep = RF.sample_labels(600, ei, ej, p, 99, 6)
    for s in range(6):
        # the kept indicators follow the documented uniform stream
        u = np.array([RF.uniform(99, s, a, c) for a, c in zip(ei, ej)])
        np.testing.assert_array_equal(keep[s], (u < p).astype(np.uint8))
        k = keep[s].astype(bool)
        g = sp.coo_matrix((np.ones(k.sum()), (ei[k], ej[k])), shape=(600, 600))
        nc, lab = connected_components(g, directed=False)
        mins = np.full(nc, 600)
        np.minimum.at(mins, lab, np.arange(600))
        np.testing.assert_array_equal(root[s], mins[lab])


def loss_pair(root):
    return float(root[1] == root[0])


def test_enumeration_single_edge_closed_form():
    pos = np.array([[1.0, 1.0, 1.0], [1.18, 1.0, 1.0]], np.float32)
    b, tau, L = 0.2, 0.02, 8.0
    EL, g = RF.enumerate_gradient(pos, L, b, tau, b + 10 * tau, loss_pair)
    d = float(np.float32(1.18)) - float(np.float32(1.0))
    p = 1.0 / (1.0 + np.exp(-(b - d) / tau))
    assert abs(EL - p) < 1e-14
    # dE/dx_0 = p (1 - p) dz/dx_0, dz/dx_0 = -(x0 - x1)/(tau d) = +1/tau along x
    np.testing.assert_allclose(g[0], [p * (1 - p) / tau, 0, 0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g[1], -g[0], rtol=1e-12)


def small_graph(seed):
    """A jittered 2 x 3 lattice of spacing 0.3: 7 axis pairs (p ~ 0.7 at b = 0.32) and 4
    diagonals (p ~ 0.007) within r_c = b + 10 tau = 0.52; 11 candidate edges."""
    rng = np.random.default_rng(seed)
    g = np.array([[i * 0.3, j * 0.3, 0.0] for i in range(2) for j in range(3)])
    return (2.0 + g + rng.uniform(-0.02, 0.02, g.shape)).astype(np.float32)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_enumerated_gradient_matches_finite_differences(seed):
    pos = small_graph(seed)
    L, b, tau = 8.0, 0.32, 0.02
    r_c = b + 10 * tau
    lossf = lambda root: RF.loss_sum_sq(root, 2)
    ei, ej, _ = RF.candidate_edges(pos, L, r_c)
    assert 2 <= ei.shape[0] <= 12
    EL, g = RF.enumerate_gradient(pos, L, b, tau, r_c, lossf)
    for i in range(pos.shape[0]):
        for a in range(3):
            h = 2e-4
            p1, p2 = pos.copy(), pos.copy()
            p1[i, a] = np.float32(float(p1[i, a]) + h)
            p2[i, a] = np.float32(float(p2[i, a]) - h)
            e1, e2, _ = RF.candidate_edges(p1, L, r_c)
            e3, e4, _ = RF.candidate_edges(p2, L, r_c)
            assert e1.shape == ei.shape and e3.shape == ei.shape   # edge set unchanged
            den = float(p1[i, a]) - float(p2[i, a])
            fd = (RF.expected_loss(p1, L, b, tau, r_c, lossf) -
                  RF.expected_loss(p2, L, b, tau, r_c, lossf)) / den
            assert abs(fd - g[i, a]) <= 1e-3 * max(abs(g).max(), 1e-9), (i, a, fd, g[i, a])


@pytest.mark.parametrize("baseline", ["loo", "none"])
def test_estimator_is_unbiased(baseline):
    pos = small_graph(4)
    L, b, tau = 8.0, 0.32, 0.02
    r_c = b + 10 * tau
    lossf = lambda root: RF.loss_sum_sq(root, 2)
    _, g_exact = RF.enumerate_gradient(pos, L, b, tau, r_c, lossf)
    ei, ej, d2 = RF.candidate_edges(pos, L, r_c)
    delta, d = RF.edge_geometry(pos, L, ei, ej)
    p = RF.edge_prob(d2, b, tau)
    K, reps = 16, 400
    ests = []
    for rep in range(reps):
        root, keep = RF.sample_labels(pos.shape[0], ei, ej, p, 1000 + rep, K)
        losses = [lossf(root[s]) for s in range(K)]
        ests.append(RF.score_gradient(pos.shape[0], ei, ej, delta, d, p, tau, keep, losses,
                                      baseline))
    ests = np.array(ests)
    mean = ests.mean(axis=0)
    se = ests.std(axis=0, ddof=1) / np.sqrt(reps)
    z = np.abs(mean - g_exact) / np.maximum(se, 1e-12)
    assert np.all(z < 4.5), z.max()


# --- the paper's own Bernoulli form, p = sigmoid(alpha (b^2 - d^2) / b^2) -------------------

def test_quadratic_probability_closed_forms():
    b, alpha = 0.25, 3.0
    p = RF.edge_prob_quadratic(np.array([b * b, 0.0, 2 * b * b]), b, alpha)
    assert p[0] == 0.5                                   # z = 0 at d = b
    assert abs(p[1] - 1.0 / (1.0 + np.exp(-alpha))) < 1e-15   # z = alpha at d = 0
    assert abs(p[2] - 1.0 / (1.0 + np.exp(alpha))) < 1e-15    # z = -alpha at d = b sqrt 2


def test_quadratic_single_edge_closed_form():
    pos = np.array([[1.0, 1.0, 1.0], [1.18, 1.0, 1.0]], np.float32)
    b, alpha, L = 0.2, 2.0, 8.0
    EL, g = RF.enumerate_gradient(pos, L, b, None, 0.5, loss_pair, alpha=alpha)
    d = float(np.float32(1.18)) - float(np.float32(1.0))
    p = 1.0 / (1.0 + np.exp(-alpha * (b * b - d * d) / (b * b)))
    assert abs(EL - p) < 1e-14
    # dz/dx_0 = -2 alpha (x0 - x1) / b^2 = +2 alpha d / b^2 along x
    np.testing.assert_allclose(g[0], [p * (1 - p) * 2 * alpha * d / (b * b), 0, 0],
                               rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g[1], -g[0], rtol=1e-12)


@pytest.mark.parametrize("seed", [1, 2])
def test_quadratic_enumerated_gradient_matches_finite_differences(seed):
    pos = small_graph(seed)
    L, b, alpha, r_c = 8.0, 0.32, 3.0, 0.55   # 11 edges: axis pairs and diagonals
    lossf = lambda root: RF.loss_sum_sq(root, 2)
    ei, ej, _ = RF.candidate_edges(pos, L, r_c)
    assert 2 <= ei.shape[0] <= 12
    EL, g = RF.enumerate_gradient(pos, L, b, None, r_c, lossf, alpha=alpha)
    for i in range(pos.shape[0]):
        for a in range(3):
            h = 2e-4
            p1, p2 = pos.copy(), pos.copy()
            p1[i, a] = np.float32(float(p1[i, a]) + h)
            p2[i, a] = np.float32(float(p2[i, a]) - h)
            den = float(p1[i, a]) - float(p2[i, a])
            fd = (RF.expected_loss(p1, L, b, None, r_c, lossf, alpha=alpha) -
                  RF.expected_loss(p2, L, b, None, r_c, lossf, alpha=alpha)) / den
            assert abs(fd - g[i, a]) <= 1e-3 * max(abs(g).max(), 1e-9), (i, a, fd, g[i, a])


def test_quadratic_estimator_is_unbiased():
    pos = small_graph(4)
    L, b, alpha, r_c = 8.0, 0.32, 3.0, 0.55
    lossf = lambda root: RF.loss_sum_sq(root, 2)
    _, g_exact = RF.enumerate_gradient(pos, L, b, None, r_c, lossf, alpha=alpha)
    ei, ej, d2 = RF.candidate_edges(pos, L, r_c)
    delta, d = RF.edge_geometry(pos, L, ei, ej)
    p = RF.edge_prob_quadratic(d2, b, alpha)
    c = RF.dz_factor(d, b, alpha=alpha)
    K, reps = 16, 400
    ests = []
    for rep in range(reps):
        root, keep = RF.sample_labels(pos.shape[0], ei, ej, p, 3000 + rep, K)
        losses = [lossf(root[s]) for s in range(K)]
        ests.append(RF.score_gradient(pos.shape[0], ei, ej, delta, d, p, None, keep, losses,
                                      "loo", c=c))
    ests = np.array(ests)
    se = ests.std(axis=0, ddof=1) / np.sqrt(reps)
    z = np.abs(ests.mean(axis=0) - g_exact) / np.maximum(se, 1e-12)
    assert np.all(z < 4.5), z.max()


def test_coincident_pair_gradient_is_finite_and_matches_central_differences():
    """Two particles at one point: d = 0 has no direction, and the distance form's estimator
    gives that edge no gradient.  Central differences with a dyadic step see the same: moving
    either particle by +-h gives the same d = h on both sides, so that edge's part of E[L]
    cancels exactly."""
    pos = np.array([[2.0, 2.0, 2.0], [2.0, 2.0, 2.0], [2.3, 2.0, 2.0], [2.0, 2.3, 2.0]],
                   np.float32)
    L, b, tau = 8.0, 0.32, 0.02
    r_c = b + 10 * tau
    lossf = lambda root: RF.loss_sum_sq(root, 2)
    ei, ej, d2 = RF.candidate_edges(pos, L, r_c)
    assert ei.shape[0] == 6 and d2.min() == 0.0
    EL, g = RF.enumerate_gradient(pos, L, b, tau, r_c, lossf)
    assert np.isfinite(g).all()
    h = 2.0 ** -12
    for i in range(pos.shape[0]):
        for a in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, a] += np.float32(h)
            p2[i, a] -= np.float32(h)
            den = float(p1[i, a]) - float(p2[i, a])
            assert den == 2 * h
            fd = (RF.expected_loss(p1, L, b, tau, r_c, lossf) -
                  RF.expected_loss(p2, L, b, tau, r_c, lossf)) / den
            assert abs(fd - g[i, a]) <= 1e-3 * max(abs(g).max(), 1e-9), (i, a, fd, g[i, a])
    # the estimator on sampled graphs stays finite too
    delta, d = RF.edge_geometry(pos, L, ei, ej)
    p = RF.edge_prob(d2, b, tau)
    root, keep = RF.sample_labels(4, ei, ej, p, 7, 16)
    losses = [lossf(r) for r in root]
    est = RF.score_gradient(4, ei, ej, delta, d, p, tau, keep, losses, "loo")
    assert np.isfinite(est).all()
