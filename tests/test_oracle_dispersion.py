"""Pins of the oracle's decoration (decorated frozen assignment, paper Sec. 3.1): the
position dispersion of a group and its gradient with memberships frozen.

Closed forms (two particles, a cubic block), invariance under a periodic shift across the
box edge, central finite differences of the full function (centre of mass recomputed from
the positions), and the zero sum of the gradient over a group.
"""
import math

import numpy as np

import oracle


def test_two_particles_closed_form():
    a = 0.3
    pos = np.array([[5.0 + a, 5.0, 5.0], [5.0 - a, 5.0, 5.0]])
    s = oracle.group_dispersion(pos, np.array([0, 0]), np.array([2]), np.array([[5.0, 5.0, 5.0]]),
                                10.0)
    # |d|^2 sums to 2 a^2 over 3 * 2 components
    assert math.isclose(s[0], a / math.sqrt(3.0), rel_tol=1e-15)


def _block(k, h, c):
    g = (np.arange(k) - (k - 1) / 2.0) * h
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + np.asarray(c)


def test_cubic_block_closed_form_and_singletons():
    k, h = 4, 0.25
    pos = _block(k, h, (3.0, 4.0, 5.0))
    n = k ** 3
    gid = np.zeros(n, np.int64)
    s = oracle.group_dispersion(pos, gid, np.array([n]), np.array([[3.0, 4.0, 5.0]]), 10.0)
    # per axis the population variance of k equally spaced values is h^2 (k^2 - 1) / 12
    assert math.isclose(s[0], h * math.sqrt((k * k - 1) / 12.0), rel_tol=1e-13)
    one = oracle.group_dispersion(pos[:1], np.array([0]), np.array([1]), pos[:1], 10.0)
    assert one[0] == 0.0


def test_periodic_shift_across_the_edge():
    L = 8.0
    rng = np.random.default_rng(3)
    pos = np.array([2.0, 3.0, 4.0]) + 0.4 * rng.standard_normal((50, 3))
    com = pos.mean(axis=0)
    gid = np.zeros(50, np.int64)
    s0 = oracle.group_dispersion(pos, gid, np.array([50]), com[None], L)
    shift = np.array([-2.0, 5.5, 4.0])  # x wraps below 0, y and z above L
    s1 = oracle.group_dispersion(np.mod(pos + shift, L), gid, np.array([50]),
                                 np.mod(com + shift, L)[None], L)
    assert math.isclose(s0[0], s1[0], rel_tol=1e-12)


def _com(pos, gid, G, L):
    """Group centres: members unwrapped about the first member by minimum image, averaged."""
    com = np.zeros((G, 3))
    for g in range(G):
        x = pos[gid == g]
        d = x - x[0]
        d = np.where(d > L / 2, d - L, np.where(d < -L / 2, d + L, d))
        com[g] = np.mod(x[0] + d.mean(axis=0), L)
    return com


def test_gradient_matches_central_differences_and_sums_to_zero():
    L = 6.0
    rng = np.random.default_rng(11)
    a = np.array([0.2, 3.0, 5.9]) + 0.3 * rng.standard_normal((12, 3))  # straddles x = 0, z = L
    b = np.array([3.0, 3.0, 3.0]) + 0.2 * rng.standard_normal((7, 3))
    pos = np.mod(np.concatenate([a, b]), L)
    gid = np.array([0] * 12 + [1] * 7)
    sizes = np.array([12, 7])
    w = np.array([0.7, -1.3])  # upstream gradient

    def f(p):
        return float(np.dot(w, oracle.group_dispersion(p, gid, sizes, _com(p, gid, 2, L), L)))

    com = _com(pos, gid, 2, L)
    sig = oracle.group_dispersion(pos, gid, sizes, com, L)
    grad = oracle.dispersion_backward(pos, gid, sizes, com, sig, w, L)
    eps = 1e-6
    for i in (0, 5, 11, 12, 18):
        for c in range(3):
            p1, p0 = pos.copy(), pos.copy()
            p1[i, c] += eps
            p0[i, c] -= eps
            fd = (f(p1) - f(p0)) / (2 * eps)
            assert math.isclose(grad[i, c], fd, rel_tol=1e-6, abs_tol=1e-9), (i, c, grad[i, c], fd)
    for g in range(2):
        assert np.allclose(grad[gid == g].sum(axis=0), 0.0, atol=1e-12)
