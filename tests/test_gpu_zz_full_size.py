"""Full size: the 512^3 Zel'dovich box with 50,000 NFW clumps that bench.py measures, run in
the same launch configuration (default tuning, helper stream when the package made one), and
compared, label by label, group by group, with the oracle run on the whole box (its
multi-threaded form, pinned to the serial one in test_oracle_par.py), and again through the
streaming mode in 16 z-slabs.  Collected last: it
takes about a minute, most of it drawing the box and running the oracle.  The same pipeline
at 1024^3 runs only when FOF_TEST_1024=1 is set, checked there by properties at any size
and a 16.8M-particle slab against the oracle."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import com_close, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_full_size_zeldovich_nfw_512():
    """Every label, group id, size and centre of mass of all 134,217,728 particles."""
    from gpu_util import compare_with_oracle

    box = W.make(2)
    say(f"full size {box.name}: oracle on n={box.n}")
    ref_root, _ = oracle.fof_par(box.pos, box.L, box.b)
    say("oracle done; GPU")
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, root_ref=ref_root)
    check_stream(box, ref_root)


def check_stream(box, ref_root, nslab=16):
    """Streaming labels in 16 z-slabs: bit-exact to the whole-box labels, with a workspace
    at most a quarter of the in-core plan's."""
    import torch
    from paper_2510_26851_amd import Plan, Stream

    say(f"streaming in {nslab} slabs")
    t = torch.from_numpy(box.pos).cuda()
    st = Stream(t, box.L, box.b, nslab=nslab)
    root = st.labels()
    torch.cuda.synchronize()
    assert st.status() == 0
    np.testing.assert_array_equal(root.cpu().numpy(), ref_root)
    in_core = Plan([box.n], [(box.L, box.b)], device=t.device).ws_bytes
    say(f"stream workspace {st.ws_bytes / 1e9:.2f} GB, in core {in_core / 1e9:.2f} GB")
    assert st.ws_bytes <= in_core / 4


@pytest.mark.skipif(os.environ.get("FOF_TEST_1024") != "1",
                    reason="the 1024^3 box takes minutes and about 100 GB of host memory to "
                           "draw and index; set FOF_TEST_1024=1 to run it")
def test_full_size_zeldovich_nfw_1024():
    """1024^3 particles (1.07e9, int32 indices near their limit, 2^30 cells: the
    two-level bucketed binning) with 400,000 NFW clumps, in one box on one GPU."""
    check_full_size(W.make(5, progress=say), whole_box_oracle=False)


def check_slab(box, root, cnt, rank, com, z0, width):
    """Every component that lies inside the slab z0 <= z < z0 + width, more than b from both
    of its faces, against the oracle run on the slab alone (in a periodic box padded to
    width + 2 along z, so nothing links across the cut): such a component is the same set in
    the slab as in the whole box, since every particle outside the slab is more than b away
    from each of its members along z."""
    z = box.pos[:, 2].astype(np.float64)
    sel = np.nonzero((z >= z0) & (z < z0 + width))[0]          # ascending original indices
    sub = np.ascontiguousarray(box.pos[sel])
    assert z0 == float(np.float32(z0)) and width <= z0
    sub[:, 2] -= np.float32(z0)        # exact (z0 <= z < 2 z0), so every distance is unchanged
    Lpad = (box.L[0], box.L[1], float(width) + 2.0)
    say(f"slab oracle: {sel.size} particles")
    oroot, _ = oracle.fof(sub, Lpad, box.b)
    oroot = oroot.astype(np.int64)
    zs = z[sel] - z0
    margin = box.b * 1.001
    edge = (zs < margin) | (zs >= width - margin)
    touched = np.bincount(oroot[edge], minlength=sel.size) > 0
    inner = ~touched[oroot]                                     # members of interior components
    assert inner.mean() > 0.5
    # labels: the smallest original index of the component (ascending map local -> original)
    np.testing.assert_array_equal(root[sel[inner]], sel[oroot[inner]])
    osize = np.bincount(oroot[inner], minlength=sel.size)
    lab = np.nonzero(osize)[0]
    np.testing.assert_array_equal(cnt[sel[lab]], osize[lab])   # no member outside the slab
    ref = oracle.groups(sub, oroot.astype(np.int32), Lpad, box.min_size)
    glab = np.nonzero(np.bincount(oroot, minlength=sel.size) >= box.min_size)[0]
    keep = ~touched[glab]
    spacing = float(box.L[0]) / round(box.n ** (1 / 3))
    gcom = com[rank[sel[glab[keep]]]]
    rcom = ref["com"][:ref["n_groups"]][keep].copy()
    rcom[:, 2] += z0
    rcom[:, 2] = np.mod(rcom[:, 2], box.L[2])
    assert com_close(gcom, rcom, box.L, spacing)
    say(f"slab: {lab.size} interior components, {int(keep.sum())} groups")


def check_full_size(box, whole_box_oracle=True):
    import torch
    from paper_2510_26851_amd import Plan, trim

    n = box.n
    say(f"full size {box.name}: n={n}")
    dev = torch.device("cuda:0")
    plan = Plan([n], [(box.L, box.b)], device=dev)
    plan.build_grid(torch.from_numpy(box.pos).to(dev))
    root = plan.link()
    res = trim(plan.groups(box.min_size))
    torch.cuda.synchronize()
    assert plan.status() == 0
    say("linked")
    del plan
    root = root.cpu().numpy()
    gid = res["group_id"].cpu().numpy()
    sizes = res["sizes"].cpu().numpy()
    com = res["com"].cpu().numpy()
    say("properties")
    # labels: each particle's label is a member index no larger than its own, and a fixed point
    assert np.all(root <= np.arange(n)) and np.all(root[root] == root)
    cnt = np.bincount(root, minlength=n)
    kept = np.nonzero(cnt >= box.min_size)[0]     # ascending label = group order
    assert res["n_groups"] == kept.size > 0
    np.testing.assert_array_equal(sizes, cnt[kept])
    rank = np.full(n, -1, np.int64)
    rank[kept] = np.arange(kept.size)
    np.testing.assert_array_equal(gid, rank[root])
    width = 64.0 * (512.0 / box.L[0]) ** 2                     # about 16.8M particles
    check_slab(box, root, cnt, rank, com, 0.375 * box.L[2], width)
    if not whole_box_oracle:
        return
    say("oracle index")
    idx = oracle.Index(box.pos, box.L, box.b)
    rng = np.random.default_rng(2026)
    in_groups = np.nonzero(cnt[root] >= box.min_size)[0]
    seeds = np.concatenate([rng.choice(n, 100, replace=False),
                            rng.choice(in_groups, 100, replace=False)])
    spacing = float(box.L[0]) / round(n ** (1 / 3))
    for s in seeds:
        mem = idx.component(int(s))               # sorted original indices
        assert root[s] == mem[0], s
        assert cnt[mem[0]] == mem.size, s         # with root[s] == mem[0]: the same set
        assert np.all(root[mem] == mem[0]), s
        if mem.size >= box.min_size:
            sub = box.pos[mem]
            ref = oracle.groups(sub, np.zeros(mem.size, np.int32), box.L, 1)
            assert ref["n_groups"] == 1
            assert com_close(com[rank[mem[0]]][None], ref["com"], box.L, spacing), s
    idx.close()


def test_zeldovich_256_against_the_full_oracle():
    """The 256^3 Zel'dovich box (16.8M particles): every label, group id, size and centre of
    mass against the oracle run on the whole box."""
    from gpu_util import compare_with_oracle

    box = W.make(1)
    say(f"full oracle comparison {box.name}: n={box.n}")
    ref_root, _ = oracle.fof_par(box.pos, box.L, box.b)
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, root_ref=ref_root)
