"""Batches of independent periodic boxes in one plan (one set of launches).

Labels are global indices into the concatenated arrays, so box k's labels minus its offset
must equal the oracle's labels of that box alone, bit for bit; group ids are numbered
across the batch in ascending label order (box by box).
"""
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


def run_batch(boxes, min_size, tune=None):
    import torch
    from paper_2510_26851_amd import Plan, trim

    dev = torch.device("cuda:0")
    counts = [bx.n for bx in boxes]
    pos = torch.from_numpy(np.concatenate([bx.pos for bx in boxes])).to(dev)
    plan = Plan(counts, [(bx.L, bx.b) for bx in boxes], device=dev, tune=tune)
    plan.build_grid(pos)
    root = plan.link()
    res = trim(plan.groups(min_size))
    torch.cuda.synchronize()
    assert plan.status() == 0
    return root.cpu().numpy(), {k: (v.cpu().numpy() if hasattr(v, "cpu") else v)
                                for k, v in res.items()}


def check_against_oracle(boxes, root, res, min_size, which):
    offs = np.concatenate([[0], np.cumsum([bx.n for bx in boxes])])
    gbase = 0
    gid = res["group_id"]
    # group ids are global: count the groups of every box in order
    per_box_groups = []
    for k, bx in enumerate(boxes):
        r = root[offs[k]:offs[k + 1]] - offs[k]
        assert np.all((r >= 0) & (r < bx.n))
        per_box_groups.append(None)
    for k in range(len(boxes)):
        bx = boxes[k]
        sl = slice(offs[k], offs[k + 1])
        if k in which:
            ref, _ = oracle.fof_par(bx.pos, bx.L, bx.b)
            np.testing.assert_array_equal(root[sl] - offs[k], ref)
            g = oracle.groups(bx.pos, ref, bx.L, min_size)
            local = gid[sl]
            kept = local >= 0
            np.testing.assert_array_equal(kept, g["group_id"] >= 0)
            if kept.any():
                np.testing.assert_array_equal(local[kept] - local[kept].min(), g["group_id"][kept])
                first = local[kept].min()
                G = g["n_groups"]
                np.testing.assert_array_equal(res["sizes"][first:first + G], g["sizes"])
                spacing = (np.prod(bx.L) / bx.n) ** (1.0 / 3.0)
                assert com_close(res["com"][first:first + G], g["com"], bx.L, spacing)


def test_small_batch_mixed_sizes():
    rng = np.random.default_rng(5)
    boxes = []
    for k, n in enumerate([1, 50, 700, 4096, 0, 20000, 333, 12000]):
        if n == 0:
            boxes.append(W.Box(np.zeros((0, 3), np.float32), (5.0,) * 3, 0.4, 2, name="empty"))
            continue
        L = 2.0 * max(n, 8) ** (1 / 3)
        pos = W.clumpy_box(n, L, max(1, n // 800), 100 + k) if n > 1 else \
            W.uniform_box(1, (L,) * 3, 3)
        boxes.append(W.Box(pos, (L, L, L), W.linking_length(0.2, L, max(n, 8)), 5))
    say("batch of 8 mixed boxes")
    root, res = run_batch(boxes, 5)
    check_against_oracle(boxes, root, res, 5, which=set(range(len(boxes))))


@pytest.mark.slow
def test_config4_batch_of_256_boxes():
    """All 256 boxes of the batched workload in one plan, every box against the oracle."""
    boxes = W.config4()
    n = sum(bx.n for bx in boxes)
    say(f"config4: {len(boxes)} boxes, {n} particles")
    root, res = run_batch(boxes, 20)
    check_against_oracle(boxes, root, res, 20, set(range(len(boxes))))
    # labels are canonical everywhere: root[root[i]] == root[i] and root[i] <= i
    idx = np.arange(root.shape[0])
    assert np.all(root <= idx) and np.all(root[root] == root)


def test_batched_equals_looped():
    import torch
    from paper_2510_26851_amd import find_groups

    boxes = W.config4(nbox=12, n_lo=16 ** 3, n_hi=48 ** 3)
    say(f"batched vs looped on {len(boxes)} boxes")
    root, res = run_batch(boxes, 20)
    offs = np.concatenate([[0], np.cumsum([bx.n for bx in boxes])])
    for k, bx in enumerate(boxes):
        r1, g1 = find_groups(torch.from_numpy(bx.pos).cuda(), bx.L, bx.b, 20)
        np.testing.assert_array_equal(root[offs[k]:offs[k + 1]] - offs[k], r1.cpu().numpy())


def test_autotuned_batch_equals_the_oracle(tmp_path):
    """The autotuner's choice for a batch (cell size relative to each box's spacing, dense
    threshold, block shape) leaves every box's labels and groups equal to the oracle's."""
    import torch
    from paper_2510_26851_amd.tune import autotune_batch

    boxes = W.config4(nbox=24, n_lo=16 ** 3, n_hi=64 ** 3)
    counts = [bx.n for bx in boxes]
    pos = torch.from_numpy(np.concatenate([bx.pos for bx in boxes])).cuda()
    say(f"autotuning a batch of {len(boxes)} boxes")
    tune = autotune_batch(pos, counts, [(bx.L, bx.b) for bx in boxes], 20,
                          cache=str(tmp_path / "tune.json"), reps=1, log=say)
    assert set(tune) >= {"cell_factor", "dense_threshold"}
    say(f"tuned: {tune}")
    root, res = run_batch(boxes, 20, tune=tune)
    check_against_oracle(boxes, root, res, 20, set(range(len(boxes))))
