"""Pins of the oracle's six-dimensional sub-halo pass (paper Sec. 2, sub-halo finding): its
reduction to the three-dimensional pass when velocities carry no weight (against the C cell-
list oracle), a velocity split in closed form, scale invariance, the minimum image, host
independence and hand cases."""
import numpy as np

import oracle
import workloads as W

INF = np.inf


def _hosts(seed=3, L=24.0, b=0.2):
    pos, vel = W.phase_space_hosts(5, L, seed, members=(30, 200), n_background=4000)
    root, _ = oracle.fof(pos, L, b)
    g = oracle.groups(pos, root, L, 20)
    return pos, vel, g["group_id"], g["n_groups"], L, b, root


def test_without_velocity_weight_each_host_is_its_own_fof_group():
    pos, vel, gid, G, L, b, root = _hosts()
    assert G >= 5
    one = np.ones(G)
    sub = oracle.subhalos(pos, vel, gid, one, np.full(G, INF), b, L)
    inh = gid >= 0
    np.testing.assert_array_equal(sub[inh], root[inh])
    assert np.all(sub[~inh] == -1)


def test_without_velocity_weight_a_shorter_length_matches_the_finer_fof():
    pos, vel, gid, G, L, b, _ = _hosts(seed=5)
    fine, _ = oracle.fof(pos, L, 0.1)          # every 0.1-component lies inside one host or none
    sub = oracle.subhalos(pos, vel, gid, np.ones(G), np.full(G, INF), 0.1, L)
    inh = gid >= 0
    np.testing.assert_array_equal(sub[inh], fine[inh])
    assert np.unique(sub[inh]).size > G       # the finer pass really splits hosts


def test_two_streams_at_one_place_split_by_velocity():
    # two chains of particles 0.05 apart along x, 0.01 apart from each other, moving at +-10
    k = 40
    x = np.zeros((2 * k, 3))
    x[:k, 0] = 5.0 + 0.05 * np.arange(k)
    x[k:, 0] = 5.0 + 0.05 * np.arange(k)
    x[:, 1] = 5.0
    x[k:, 1] += 0.01
    x[:, 2] = 5.0
    perm = np.random.default_rng(0).permutation(2 * k)
    pos = x[perm].astype(np.float32)
    v = np.zeros((2 * k, 3), np.float32)
    v[:k, 0], v[k:, 0] = 10.0, -10.0
    vel = v[perm]
    gid = np.zeros(2 * k, np.int32)
    sub = oracle.subhalos(pos, vel, gid, [0.04], [1.0], 1.0, 20.0)
    a = np.nonzero(perm < k)[0]
    b = np.nonzero(perm >= k)[0]
    assert np.all(sub[a] == a.min()) and np.all(sub[b] == b.min())
    # with no velocity weight the two streams are one sub-halo
    sub1 = oracle.subhalos(pos, vel, gid, [0.04], [INF], 1.0, 20.0)
    assert np.all(sub1 == 0)


def test_scaling_velocities_with_their_factor_changes_nothing():
    pos, vel, gid, G, L, _, _ = _hosts(seed=7)
    rng = np.random.default_rng(1)
    nx = rng.uniform(0.02, 0.06, G)
    nv = rng.uniform(0.5, 2.0, G)
    s1 = oracle.subhalos(pos, vel, gid, nx, nv, 1.0, L)
    s2 = oracle.subhalos(pos, vel * np.float32(2.0), gid, nx, nv * 4.0, 1.0, L)
    np.testing.assert_array_equal(s1, s2)
    inh = gid >= 0
    assert np.unique(s1[inh]).size > G        # velocities split some hosts


def test_hosts_are_independent_and_outsiders_get_minus_one():
    pos, vel, gid, G, L, _, _ = _hosts(seed=9)
    nx, nv = np.full(G, 0.04), np.full(G, 1.0)
    full = oracle.subhalos(pos, vel, gid, nx, nv, 1.0, L)
    for g in range(G):
        m = np.nonzero(gid == g)[0]
        alone = oracle.subhalos(pos[m], vel[m], np.zeros(m.size, np.int32), nx[g:g + 1],
                                nv[g:g + 1], 1.0, L)
        np.testing.assert_array_equal(full[m], m[alone])
    # a host split in two by its group ids never links across the split
    g0 = np.nonzero(gid == 0)[0]
    gid2 = gid.copy()
    gid2[g0[::2]] = G
    sp = oracle.subhalos(pos, vel, gid2, np.append(nx, 0.04), np.append(nv, 1.0), 1.0, L)
    assert not np.intersect1d(sp[g0[::2]], sp[g0[1::2]]).size


def test_hand_cases():
    L = 10.0
    # a chain 2 - 0 - 1 along x: 0.15 apart, ends 0.3 apart; one component labelled 0
    pos = np.array([[5.15, 5, 5], [5.3, 5, 5], [5.0, 5, 5]], np.float32)
    vel = np.zeros((3, 3), np.float32)
    gid = np.zeros(3, np.int32)
    np.testing.assert_array_equal(oracle.subhalos(pos, vel, gid, [1.0], [1.0], 0.2, L), [0, 0, 0])
    # the same chain across the box face (minimum image)
    pos2 = np.array([[0.05, 5, 5], [0.2, 5, 5], [9.9, 5, 5]], np.float32)
    np.testing.assert_array_equal(oracle.subhalos(pos2, vel, gid, [1.0], [1.0], 0.2, L), [0, 0, 0])
    # velocity term: |dv|^2 / 4 = 0.0225 + 0.0225 < 0.2^2 fails, so the middle link breaks
    vel3 = np.array([[0, 0, 0], [0.3, 0, 0], [0, 0, 0]], np.float32)
    # pair (0,2): 0.0225 + 0 < 0.04 links; pair (0,1): 0.0225 + 0.0225 = 0.045 does not
    np.testing.assert_array_equal(oracle.subhalos(pos, vel3, gid, [1.0], [4.0], 0.2, L),
                                  [0, 1, 0])
    # non-positive factors leave singletons; particles outside hosts get -1
    np.testing.assert_array_equal(oracle.subhalos(pos, vel, gid, [0.0], [1.0], 0.2, L), [0, 1, 2])
    np.testing.assert_array_equal(
        oracle.subhalos(pos, vel, np.array([0, -1, 0], np.int32), [1.0], [1.0], 0.2, L),
        [0, -1, 0])
