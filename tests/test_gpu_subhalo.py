"""Six-dimensional sub-halo pass (paper Sec. 2, sub-halo finding) on the GPU against the
oracle: hosts from each side's own three-dimensional pass, then every sub-halo label compared
exactly (the phase-space predicate is evaluated in FP64 in the same order on both sides)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run(pos, vel, L, b, min_size, nx, nv, b6):
    import torch
    from paper_2510_26851_amd import Plan, trim

    dev = torch.device("cuda:0")
    plan = Plan([pos.shape[0]], [(L, b)], device=dev)
    tp = torch.from_numpy(pos).to(dev)
    tv = torch.from_numpy(vel).to(dev)
    plan.build_grid(tp)
    plan.link()
    res = trim(plan.groups(min_size))
    G = int(res["n_groups"])
    fx = nx(G) if callable(nx) else nx
    fv = nv(G) if callable(nv) else nv
    sub = plan.subhalo(tp, tv, res["group_id"], G, res["sizes"], fx, fv, b6)
    torch.cuda.synchronize()
    assert plan.status() == 0
    return res["group_id"].cpu().numpy(), G, sub.cpu().numpy()


@pytest.mark.parametrize("seed,hosts,members,in_lds",
                         [(11, 6, (30, 400), True), (12, 3, (600, 1100), False)])
def test_subhalo_matches_oracle(seed, hosts, members, in_lds):
    """Seed 11 has hosts of at most 2048 members (whole host and union-find in LDS); seed 12
    only hosts above 2048 (tiles through LDS, union-find in HBM)."""
    L, b = 24.0, 0.2
    pos, vel = W.phase_space_hosts(hosts, L, seed, members=members, n_background=6000)
    say(f"sub-halo seed={seed} n={pos.shape[0]}")
    rng = np.random.default_rng(seed)
    fx = rng.uniform(0.02, 0.06, 4096)
    fv = rng.uniform(0.5, 2.0, 4096)
    gid, G, sub = run(pos, vel, L, b, 20, lambda G: fx[:G], lambda G: fv[:G], 1.0)
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, 20)
    assert G == ref["n_groups"] >= hosts
    np.testing.assert_array_equal(gid, ref["group_id"])
    sz = ref["sizes"][:G]
    say(f"host sizes {sz.min()}..{sz.max()}")
    assert (sz.max() <= 2048) if in_lds else (sz.min() > 2048)
    want = oracle.subhalos(pos, vel, ref["group_id"], fx[:G], fv[:G], 1.0, L)
    np.testing.assert_array_equal(sub, want)
    inh = gid >= 0
    assert np.unique(sub[inh]).size > G          # velocities split hosts


def test_subhalo_without_velocity_weight_is_the_host():
    L, b = 24.0, 0.2
    pos, vel = W.phase_space_hosts(4, L, 13, n_background=3000)
    gid, G, sub = run(pos, vel, L, b, 20, lambda G: np.ones(G), lambda G: np.full(G, np.inf), b)
    root, _ = oracle.fof(pos, L, b)
    inh = gid >= 0
    np.testing.assert_array_equal(sub[inh], root[inh])
    assert np.all(sub[~inh] == -1)


def test_subhalo_with_no_hosts():
    L, b = 24.0, 0.2
    pos = W.uniform_box(2000, (L, L, L), 14)
    vel = np.zeros_like(pos)
    gid, G, sub = run(pos, vel, L, b, 20, np.ones(1), np.ones(1), 1.0)
    assert G == 0 and np.all(sub == -1)


def test_subhalo_in_a_batch_of_two_boxes():
    """Two boxes of different sizes in one plan: each host uses its own box's minimum image,
    and hosts of different boxes never link."""
    import torch
    from paper_2510_26851_amd import Plan, trim

    b = 0.2
    boxes = [(24.0, W.phase_space_hosts(4, 24.0, 21, n_background=3000)),
             (16.0, W.phase_space_hosts(3, 16.0, 22, n_background=2000))]
    n1 = boxes[0][1][0].shape[0]
    pos = np.concatenate([p for _, (p, _) in boxes])
    vel = np.concatenate([v for _, (_, v) in boxes])
    dev = torch.device("cuda:0")
    plan = Plan([p.shape[0] for _, (p, _) in boxes], [(L, b) for L, _ in boxes], device=dev)
    tp, tv = torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev)
    plan.build_grid(tp)
    plan.link()
    res = trim(plan.groups(20))
    G = int(res["n_groups"])
    rng = np.random.default_rng(23)
    fx, fv = rng.uniform(0.02, 0.06, G), rng.uniform(0.5, 2.0, G)
    sub = plan.subhalo(tp, tv, res["group_id"], G, res["sizes"], fx, fv, 1.0)
    torch.cuda.synchronize()
    assert plan.status() == 0
    sub, gid = sub.cpu().numpy(), res["group_id"].cpu().numpy()
    refs, base, g0 = [], 0, 0
    for L, (p, v) in boxes:
        root, _ = oracle.fof(p, L, b)
        ref = oracle.groups(p, root, L, 20)
        rg = ref["group_id"].astype(np.int64)
        np.testing.assert_array_equal(gid[base:base + p.shape[0]], np.where(rg >= 0, rg + g0, -1))
        k = ref["n_groups"]
        want = oracle.subhalos(p, v, ref["group_id"], fx[g0:g0 + k], fv[g0:g0 + k], 1.0, L)
        np.testing.assert_array_equal(sub[base:base + p.shape[0]],
                                      np.where(want >= 0, want + base, -1))
        base += p.shape[0]
        g0 += k
    assert g0 == G and base == pos.shape[0] and n1 < base


def test_subhalo_sizes_that_disagree_with_the_ids():
    """Host sizes from another catalogue: a host declared larger than it is keeps every
    label exact; one declared smaller drops its extra members (label -1) and raises
    FOF_STATUS_RANGE, and the other hosts are unaffected."""
    import torch
    from paper_2510_26851_amd import Plan, trim, _lib

    L, b = 24.0, 0.2
    pos, vel = W.phase_space_hosts(4, L, 31, n_background=3000)
    dev = torch.device("cuda:0")
    plan = Plan([pos.shape[0]], [(L, b)], device=dev)
    tp, tv = torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev)
    plan.build_grid(tp)
    plan.link()
    res = trim(plan.groups(20))
    G = int(res["n_groups"])
    gid = res["group_id"].cpu().numpy()
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, 20)
    np.testing.assert_array_equal(gid, ref["group_id"])
    nx, nv = np.full(G, 0.04), np.ones(G)
    want = oracle.subhalos(pos, vel, ref["group_id"], nx, nv, 1.0, L)
    big = res["sizes"].clone()
    big[0] += 5
    sub = plan.subhalo(tp, tv, res["group_id"], G, big, nx, nv, 1.0).cpu().numpy()
    torch.cuda.synchronize()
    assert plan.status() == 0
    np.testing.assert_array_equal(sub, want)
    small = res["sizes"].clone()
    small[0] -= 3
    sub = plan.subhalo(tp, tv, res["group_id"], G, small, nx, nv, 1.0).cpu().numpy()
    torch.cuda.synchronize()
    assert plan.status() & _lib.FOF_STATUS_RANGE
    h0 = gid == 0
    assert np.sum(sub[h0] == -1) == 3
    np.testing.assert_array_equal(sub[~h0], want[~h0])
    # a negative size: that host's members are dropped (flagged), the host ranges after it
    # do not move backwards, and every other host stays exact
    neg = res["sizes"].clone()
    neg[1] = -7
    plan.build_grid(tp)   # clears the status word
    sub = plan.subhalo(tp, tv, res["group_id"], G, neg, nx, nv, 1.0).cpu().numpy()
    torch.cuda.synchronize()
    assert plan.status() & _lib.FOF_STATUS_RANGE
    h1 = gid == 1
    assert np.all(sub[h1] == -1)
    np.testing.assert_array_equal(sub[~h1], want[~h1])
