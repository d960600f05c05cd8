"""The whole pipeline (build + link + groups) for a batch of boxes captured in one hipGraph
and replayed; the eager labels equal the oracle's box by box, and every replay must equal
the eager result (labels, group ids, sizes bit-exact).
The library clears its buffers with fill kernels, never hipMemsetAsync."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_batched_pipeline_graph_replays_match_eager():
    import torch
    from paper_2510_26851_amd import Plan

    boxes = W.config4(nbox=24, n_lo=16 ** 3, n_hi=64 ** 3)
    say(f"hipGraph capture of {len(boxes)} boxes")
    dev = torch.device("cuda:0")
    counts = [bx.n for bx in boxes]
    n = sum(counts)
    pos = torch.from_numpy(np.concatenate([bx.pos for bx in boxes])).to(dev)
    plan = Plan(counts, [(bx.L, bx.b) for bx in boxes], device=dev)
    out = dict(group_id=torch.empty(n, dtype=torch.int32, device=dev),
               n_groups=torch.empty(1, dtype=torch.int32, device=dev),
               sizes=torch.empty(n, dtype=torch.int32, device=dev),
               com=torch.empty((n, 3), dtype=torch.float64, device=dev))
    root = torch.empty(n, dtype=torch.int32, device=dev)

    def step():
        plan.build_grid(pos)
        plan.link(root)
        plan.groups(20, out=out)

    step()
    torch.cuda.synchronize()
    ref = (root.clone(), out["group_id"].clone(), int(out["n_groups"].item()))
    refsz = out["sizes"][:ref[2]].clone()
    # the eager batch itself against the oracle, box by box (labels are batch indices)
    import oracle

    got, off = ref[0].cpu().numpy(), 0
    for bx in boxes:
        r, _ = oracle.fof(bx.pos, bx.L, bx.b)
        np.testing.assert_array_equal(got[off:off + bx.n], r + off)
        off += bx.n

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(4):
        root.fill_(-7)
        out["group_id"].fill_(-7)
        out["n_groups"].fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(root, ref[0]), rep
        assert torch.equal(out["group_id"], ref[1]), rep
        assert int(out["n_groups"].item()) == ref[2]
        assert torch.equal(out["sizes"][:ref[2]], refsz)
        # eager work between replays
        _ = (pos * 2.0).sum().item()
        assert plan.status() == 0
