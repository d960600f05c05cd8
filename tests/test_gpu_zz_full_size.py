"""Full size: the 512^3 Zel'dovich box with 50,000 NFW clumps that bench.py measures, run in
the same launch configuration (default tuning, helper stream), checked by properties that
hold at any size and, on 200 seeded particles (half of them in groups), against the oracle's
exact single-component search over the whole box.  (Collected last: it takes about two
minutes, most of it generating the box and indexing it for the oracle.)"""
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
    import torch
    from paper_2510_26851_amd import Plan, trim

    box = W.make(2)
    n = box.n
    say(f"full size {box.name}: n={n}")
    dev = torch.device("cuda:0")
    plan = Plan([n], [(box.L, box.b)], device=dev)
    plan.build_grid(torch.from_numpy(box.pos).to(dev))
    root = plan.link()
    res = trim(plan.groups(box.min_size))
    torch.cuda.synchronize()
    assert plan.status() == 0
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
    compare_with_oracle(box.pos, box.L, box.b, box.min_size)
