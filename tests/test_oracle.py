"""Pins of the CPU oracle against things other than itself (runs without a GPU).

* link predicate: hand cases in ``golden/predicate_cases.txt`` (Sec. 2 step (iv)).
* components: O(N^2) brute force + ``scipy.sparse.csgraph.connected_components`` (a library
  routine, no cell list), closed lattice cases, invariants, metamorphic permutation.
* groups: closed forms (sizes, rank order), hand centres of mass, ``math.fsum``.
* frozen backward: closed forms and central finite differences of the oracle's own forward
  with memberships frozen (Sec. 3.1).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------
# brute force (independent of the oracle's cell list and union-find)
# ------------------------------------------------------------------------------------------
def brute_labels(pos, L, b):
    """All-pairs adjacency in numpy float64 and scipy connected components, canonicalised to
    the minimum member index."""
    x = pos.astype(np.float64)
    n = x.shape[0]
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    rows, cols = [], []
    for i in range(n - 1):
        d = x[i] - x[i + 1:]
        for a in range(3):
            da = d[:, a]
            da[da > 0.5 * L[a]] -= L[a]
            da[da < -0.5 * L[a]] += L[a]
        s = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
        s = s + d[:, 2] * d[:, 2]
        j = np.nonzero(s < b * b)[0] + i + 1
        rows.append(np.full(j.shape, i))
        cols.append(j)
    rows = np.concatenate(rows) if rows else np.zeros(0, int)
    cols = np.concatenate(cols) if cols else np.zeros(0, int)
    g = sp.coo_matrix((np.ones(rows.shape[0]), (rows, cols)), shape=(n, n))
    ncomp, lab = connected_components(g, directed=False)
    mins = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(mins, lab, np.arange(n))
    return mins[lab].astype(np.int32), rows.shape[0]


def check_partition_invariants(root):
    n = root.shape[0]
    idx = np.arange(n)
    assert np.all(root <= idx)                       # label is the minimum member index
    assert np.all(root[root] == root)                # labels are fixed points
    # each label is the minimum index in its class
    mins = np.full(n, n, dtype=np.int64)
    np.minimum.at(mins, root, idx)
    assert np.all(mins[root] == root)


# ------------------------------------------------------------------------------------------
# predicate
# ------------------------------------------------------------------------------------------
def _predicate_cases():
    out = []
    with open(os.path.join(GOLDEN, "predicate_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            v = [np.float32(t) for t in tok[:6]]
            L = [float(t) for t in tok[6:9]]
            out.append((np.array(v[:3], np.float32), np.array(v[3:6], np.float32), L,
                        float(tok[9]), int(tok[10]), " ".join(tok[11:])))
    return out


@pytest.mark.parametrize("case", _predicate_cases(), ids=lambda c: c[5][:40])
def test_predicate_hand_cases(case):
    xi, xj, L, b, expect, _ = case
    assert oracle.linked(xi, xj, L, b) == bool(expect)
    assert oracle.linked(xj, xi, L, b) == bool(expect)   # symmetric


def test_predicate_float32_0p4_is_above_0p4():
    assert float(np.float32(0.4)) == 0.4000000059604645
    assert not oracle.linked(np.zeros(3, np.float32), np.array([0.4, 0, 0], np.float32), 64, 0.4)


def test_dist2_exact_dyadic():
    d2 = oracle.dist2(np.array([1.0, 2.0, 3.0], np.float32), np.array([1.5, 2.25, 3.125], np.float32),
                      10.0)
    assert d2 == 0.25 + 0.0625 + 0.015625


# ------------------------------------------------------------------------------------------
# components vs brute force
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,n,L,b", [
    (1, 500, 10.0, 0.6),
    (2, 1500, 16.0, 0.9),
    (3, 2000, (12.0, 9.0, 20.0), 0.7),
    (4, 800, 3.0, 0.35),       # n_c = 8 per axis
    (5, 300, 2.0, 0.45),       # n_c = 4
    (6, 200, 1.0, 0.4),        # n_c = 2 per axis: duplicate neighbour cells must be merged
    (7, 100, 0.9, 0.44),       # n_c = 2
    (8, 50, (0.7, 3.0, 5.0), 0.34),  # n_c = 2 on x only
])
def test_fof_matches_brute_force_uniform(seed, n, L, b):
    pos = W.uniform_box(n, np.broadcast_to(L, (3,)), seed)
    ref, nlinks = brute_labels(pos, L, b)
    got, nl = oracle.fof(pos, L, b)
    assert nl == nlinks
    np.testing.assert_array_equal(got, ref)
    check_partition_invariants(got)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_fof_matches_brute_force_clumpy(seed):
    pos = W.clumpy_box(2000, 24.0, 6, seed)
    ref, nlinks = brute_labels(pos, 24.0, 0.5)
    got, nl = oracle.fof(pos, 24.0, 0.5)
    assert nl == nlinks
    np.testing.assert_array_equal(got, ref)


def test_fof_config0_subsample_matches_brute_force():
    box = W.config0()
    # a spatial sub-box keeps the clumps; periodic wrap of the full box is kept
    pos = box.pos[:2000]
    ref, _ = brute_labels(pos, box.L, box.b)
    got, _ = oracle.fof(pos, box.L, box.b)
    np.testing.assert_array_equal(got, ref)


# ------------------------------------------------------------------------------------------
# closed cases
# ------------------------------------------------------------------------------------------
def test_lattice_below_b_is_one_group():
    pos = W.cubic_lattice(12, 0.375)           # L = 4.5, spacing 0.375 < b = 0.4
    root, nl = oracle.fof(pos, 4.5, 0.4)
    assert np.all(root == 0)
    assert nl == 3 * 12 ** 3                   # each site links to its 6 axis neighbours


def test_lattice_above_b_is_all_singletons():
    pos = W.cubic_lattice(12, 0.4375)          # L = 5.25, spacing 0.4375 > b = 0.4
    root, nl = oracle.fof(pos, 5.25, 0.4)
    np.testing.assert_array_equal(root, np.arange(pos.shape[0]))
    assert nl == 0


def test_empty_and_single():
    root, nl = oracle.fof(np.zeros((0, 3), np.float32), 10.0, 0.5)
    assert root.shape == (0,) and nl == 0
    root, nl = oracle.fof(np.array([[1, 2, 3]], np.float32), 10.0, 0.5)
    assert list(root) == [0] and nl == 0


def test_pair_across_face_and_corner_group():
    pos = np.array([[0.05, 5, 5], [9.9, 5, 5], [3, 3, 3],
                    [9.95, 9.95, 9.95], [0.05, 0.05, 0.05], [0.05, 9.95, 0.1]], np.float32)
    root, _ = oracle.fof(pos, 10.0, 0.3)
    assert list(root) == [0, 0, 2, 3, 3, 3]


def test_invalid_arguments_raise():
    pos = np.array([[1, 1, 1]], np.float32)
    for L, b in [(10.0, 0.0), (10.0, -1.0), (1.0, 0.5), (0.0, 0.1), (np.inf, 0.1)]:
        with pytest.raises(oracle.OracleError):
            oracle.fof(pos, L, b)
    with pytest.raises(oracle.OracleError):
        oracle.fof(np.array([[10.0, 1, 1]], np.float32), 10.0, 0.5)   # x == L
    with pytest.raises(oracle.OracleError):
        oracle.fof(np.array([[np.nan, 1, 1]], np.float32), 10.0, 0.5)


# ------------------------------------------------------------------------------------------
# metamorphic
# ------------------------------------------------------------------------------------------
def test_permutation_permutes_components():
    pos = W.clumpy_box(3000, 20.0, 5, 21)
    root, _ = oracle.fof(pos, 20.0, 0.5)
    perm = np.random.default_rng(0).permutation(pos.shape[0])
    root_p, _ = oracle.fof(pos[perm], 20.0, 0.5)
    # same partition: particles i, j share a label in one run iff they do in the other
    a = root[perm]
    b = root_p
    pairs = {}
    for x, y in zip(a, b):
        assert pairs.setdefault(x, y) == y
    assert len(set(pairs.values())) == len(pairs)


def test_integer_translation_keeps_partition():
    pos = W.clumpy_box(2000, 16.0, 4, 31)
    # coordinates on the 2^-10 grid so that a shift of 3 (mod L) is exact in float32
    pos = (np.round(pos.astype(np.float64) * 1024) / 1024).astype(np.float32) % np.float32(16)
    root, _ = oracle.fof(pos, 16.0, 0.45)
    sh = ((pos.astype(np.float64) + 3.0) % 16.0).astype(np.float32)
    root_s, _ = oracle.fof(sh, 16.0, 0.45)
    np.testing.assert_array_equal(root, root_s)


# ------------------------------------------------------------------------------------------
# component query (BFS) vs full run
# ------------------------------------------------------------------------------------------
def test_component_query_matches_fof():
    box = W.config0()
    root, _ = oracle.fof(box.pos, box.L, box.b)
    idx = oracle.Index(box.pos, box.L, box.b)
    rng = np.random.default_rng(5)
    for s in rng.integers(0, box.n, 40):
        mem = idx.component(int(s))
        np.testing.assert_array_equal(mem, np.nonzero(root == root[s])[0])
    idx.close()


# ------------------------------------------------------------------------------------------
# groups
# ------------------------------------------------------------------------------------------
def _com_cases():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "com_cases.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "case":
                cur = dict(name=t[1], p=[], com=None)
                cases.append(cur)
            elif t[0] == "p":
                cur["p"].append([float(v) for v in t[1:4]])
            elif t[0] == "com":
                cur["com"] = [float(v) for v in t[1:4]]
    return cases


@pytest.mark.parametrize("case", _com_cases(), ids=lambda c: c["name"])
def test_com_hand_cases(case):
    pos = np.array(case["p"], np.float32)
    root, _ = oracle.fof(pos, 64.0, 0.4)
    assert np.all(root == 0)
    g = oracle.groups(pos, root, 64.0, 2)
    assert g["n_groups"] == 1 and g["sizes"][0] == pos.shape[0]
    d = g["com"][0] - np.array(case["com"])
    d = (d + 32.0) % 64.0 - 32.0
    assert np.all(np.abs(d) < 1e-12)


def test_groups_closed_forms_and_fsum():
    box = W.config0()
    root, _ = oracle.fof(box.pos, box.L, box.b)
    g = oracle.groups(box.pos, root, box.L, box.min_size)
    labels, counts = np.unique(root, return_counts=True)
    kept = labels[counts >= box.min_size]
    assert g["n_groups"] == kept.shape[0]
    np.testing.assert_array_equal(g["sizes"], counts[counts >= box.min_size])
    rank = {r: k for k, r in enumerate(kept)}
    expect = np.array([rank.get(r, -1) for r in root], np.int32)
    np.testing.assert_array_equal(g["group_id"], expect)
    # exact-sum cross check of the unwrapped mean with math.fsum
    L = 64.0
    for k, r in enumerate(kept[:10]):
        mem = np.nonzero(root == r)[0]
        for a in range(3):
            d = [float(box.pos[i, a]) - float(box.pos[r, a]) for i in mem]
            d = [v - L if v > L / 2 else (v + L if v < -L / 2 else v) for v in d]
            c = float(box.pos[r, a]) + math.fsum(d) / len(mem)
            c = c - L if c >= L else (c + L if c < 0 else c)
            assert abs(g["com"][k, a] - c) <= 1e-12 * max(1.0, abs(c))


def test_groups_velocity_moments_closed_form():
    rng = np.random.default_rng(3)
    pos = W.cubic_lattice(4, 0.25)                        # L = 1, one group at b = 0.3
    vel = rng.standard_normal(pos.shape).astype(np.float32)
    root, _ = oracle.fof(pos, 1.0, 0.3)
    g = oracle.groups(pos, root, 1.0, 2, vel=vel)
    v = vel.astype(np.float64)
    np.testing.assert_allclose(g["vmean"][0], v.mean(axis=0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(g["sigv"][0], np.sqrt(((v - v.mean(0)) ** 2).sum() / (3 * 64)),
                               rtol=1e-14)


def test_groups_overflow_and_min_size_one():
    pos = W.cubic_lattice(4, 0.4375)                      # 64 singletons at b = 0.4
    root, _ = oracle.fof(pos, 1.75, 0.4)
    g = oracle.groups(pos, root, 1.75, 1, cap=10)
    assert g["n_groups"] == 64 and g["overflow"] and g["sizes"].shape[0] == 10
    g = oracle.groups(pos, root, 1.75, 2)
    assert g["n_groups"] == 0 and np.all(g["group_id"] == -1)


# ------------------------------------------------------------------------------------------
# frozen backward
# ------------------------------------------------------------------------------------------
def test_frozen_backward_closed_form_and_fd():
    rng = np.random.default_rng(9)
    pos = W.clumpy_box(1200, 12.0, 4, 41)
    vel = rng.standard_normal(pos.shape).astype(np.float32)
    L, b = 12.0, 0.45
    root, _ = oracle.fof(pos, L, b)
    g = oracle.groups(pos, root, L, 5, vel=vel)
    G = g["n_groups"]
    assert G >= 2
    g_com = rng.standard_normal((G, 3))
    g_sig = rng.standard_normal(G)
    g_mass = rng.standard_normal(G)
    gp, gv = oracle.frozen_backward(g["group_id"], g["sizes"], g["vmean"], g["sigv"], vel,
                                    g_mass=g_mass, g_com=g_com, g_sigv=g_sig)
    # closed forms
    gid = g["group_id"]
    kept = gid >= 0
    np.testing.assert_allclose(gp[kept], g_com[gid[kept]] / g["sizes"][gid[kept], None], rtol=0)
    assert np.all(gp[~kept] == 0) and np.all(gv[~kept] == 0)

    # central finite differences of the scalar J = sum g_com.com + g_sig.sigv + g_mass.mass
    # with memberships frozen (root held fixed), w.r.t. a few coordinates
    def J(p, v):
        gg = oracle.groups(p, root, L, 5, vel=v)
        mass = gg["sizes"].astype(np.float64)
        return float((g_com * gg["com"]).sum() + (g_sig * gg["sigv"]).sum() + (g_mass * mass).sum())

    members = np.nonzero(kept)[0]
    for i in rng.choice(members, 6, replace=False):
        for a in range(3):
            for arr, grad in ((0, gp), (1, gv)):
                h = 1e-3
                p1, v1 = pos.copy(), vel.copy()
                p2, v2 = pos.copy(), vel.copy()
                tgt1 = p1 if arr == 0 else v1
                tgt2 = p2 if arr == 0 else v2
                tgt1[i, a] = np.float32(float(tgt1[i, a]) + h)
                tgt2[i, a] = np.float32(float(tgt2[i, a]) - h)
                den = float(tgt1[i, a]) - float(tgt2[i, a])   # actually stored float32 step
                fd = (J(p1, v1) - J(p2, v2)) / den
                assert abs(fd - grad[i, a]) <= 1e-3 * max(abs(grad[i, a]), 1e-2), (i, a, arr)
