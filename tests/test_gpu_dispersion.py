"""Decorated frozen assignment (paper Sec. 3.1) through the C ABI: the per-group position
dispersion (fof_group_dispersion) and its gradient (fof_backward_dispersion) against the
FP64 oracle on the same seeded inputs."""
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


def _run(pos, L, b, min_size, cap=None):
    import torch
    from paper_2510_26851_amd import Plan

    dev = torch.device("cuda:0")
    t = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    plan = Plan([pos.shape[0]], [(L, b)], device=dev)
    plan.build_grid(t)
    plan.link()
    res = plan.groups(min_size, cap=cap)
    sig = plan.dispersion(res)
    torch.cuda.synchronize()
    return plan, t, res, sig


@pytest.mark.parametrize("seed,n,L,ncl,b,min_size", [
    (61, 20000, 24.0, 8, 0.5, 5),
    (62, 30000, 40.0, 20, 0.4, 20),
    (63, 6000, 10.0, 3, 0.35, 1),      # groups of one included: dispersion 0
    (64, 3000, 12.0, 0, 0.6, 2),       # uniform: small groups only
])
def test_dispersion_matches_oracle(seed, n, L, ncl, b, min_size):
    say(f"dispersion seed={seed} n={n} min_size={min_size}")
    pos = W.clumpy_box(n, L, ncl, seed) if ncl else W.uniform_box(n, (L,) * 3, seed)
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, min_size)
    sref = oracle.group_dispersion(pos, ref["group_id"], ref["sizes"], ref["com"], L)
    _, _, res, sig = _run(pos, L, b, min_size)
    G = int(res["n_groups"].item())
    assert G == ref["n_groups"] and G > 0
    got = sig[:G].cpu().numpy()
    np.testing.assert_allclose(got, sref, rtol=1e-9, atol=1e-12)
    if min_size <= 1:
        assert np.all(got[ref["sizes"] == 1] == 0.0)


def test_dispersion_cap_below_group_count():
    pos = W.clumpy_box(8000, 16.0, 6, 65)
    root, _ = oracle.fof(pos, 16.0, 0.45)
    ref = oracle.groups(pos, root, 16.0, 1)
    sref = oracle.group_dispersion(pos, ref["group_id"], ref["sizes"], ref["com"], 16.0)
    cap = 11
    _, _, res, sig = _run(pos, 16.0, 0.45, 1, cap=cap)
    assert int(res["n_groups"].item()) == ref["n_groups"] > cap
    np.testing.assert_allclose(sig[:cap].cpu().numpy(), sref[:cap], rtol=1e-9, atol=1e-12)


def test_dispersion_gradient_matches_oracle_and_composes():
    import torch

    L, b = 24.0, 0.5
    pos = W.clumpy_box(20000, L, 8, 66)
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, 5)
    sref = oracle.group_dispersion(pos, ref["group_id"], ref["sizes"], ref["com"], L)
    plan, t, res, sig = _run(pos, L, b, 5)
    G = int(res["n_groups"].item())
    rng = np.random.default_rng(67)
    g_sigx = rng.standard_normal(G)
    g_com = rng.standard_normal((G, 3))
    dev = t.device
    gsx = torch.from_numpy(g_sigx).to(dev)
    # dispersion gradient alone, added to zeros
    gp = torch.zeros((pos.shape[0], 3), dtype=torch.float32, device=dev)
    plan.backward_dispersion(t, res["group_id"], G, res["sizes"], res["com"], sig, gsx, gp)
    want = oracle.dispersion_backward(pos, ref["group_id"], ref["sizes"], ref["com"], sref,
                                      g_sigx, L)
    got = gp.cpu().numpy()
    scale = np.abs(want).max()
    assert scale > 0
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-5 * scale)
    # added on top of the frozen backward of the centres of mass
    gp2, _ = plan.backward(res["group_id"], G, res["sizes"],
                           g_com=torch.from_numpy(g_com).to(dev), want_vel=False)
    plan.backward_dispersion(t, res["group_id"], G, res["sizes"], res["com"], sig, gsx, gp2)
    want2 = want + oracle.frozen_backward(ref["group_id"], ref["sizes"], g_com=g_com)[0]
    np.testing.assert_allclose(gp2.cpu().numpy(), want2, rtol=0,
                               atol=1e-5 * np.abs(want2).max())


def test_dispersion_in_a_batch_of_boxes():
    import torch
    from paper_2510_26851_amd import Plan

    boxes = W.config4(nbox=6, n_lo=16 ** 3, n_hi=32 ** 3)
    dev = torch.device("cuda:0")
    counts = [bx.n for bx in boxes]
    pos = torch.from_numpy(np.concatenate([bx.pos for bx in boxes])).to(dev)
    plan = Plan(counts, [(bx.L, bx.b) for bx in boxes], device=dev)
    plan.build_grid(pos)
    plan.link()
    min_size = boxes[0].min_size  # every box of the batch uses the same cut
    res = plan.groups(min_size)
    sig = plan.dispersion(res)
    got = sig.cpu().numpy()
    # groups are numbered by label (smallest member index) over the batch: box k's groups
    # follow those of boxes 0..k-1, in the oracle's order of that box
    first = 0
    for bx in boxes:
        root, _ = oracle.fof(bx.pos, bx.L, bx.b)
        ref = oracle.groups(bx.pos, root, bx.L, min_size)
        k = ref["n_groups"]
        want = oracle.group_dispersion(bx.pos, ref["group_id"], ref["sizes"], ref["com"], bx.L)
        np.testing.assert_allclose(got[first:first + k], want, rtol=1e-9, atol=1e-12)
        first += k
    assert first == int(res["n_groups"].item())


def test_decorated_autograd_through_a_soft_histogram():
    """A loss on the soft histogram of the dispersions, differentiated through FoFDecorated,
    equals the oracle's chain: d loss / d sigx (PyTorch on the CPU, from the oracle's sigx)
    times the oracle's dispersion gradient."""
    import torch
    from paper_2510_26851_amd.autograd import fof_decorated, soft_histogram

    L, b = 24.0, 0.5
    pos = W.clumpy_box(20000, L, 8, 68)
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, 5)
    sref = oracle.group_dispersion(pos, ref["group_id"], ref["sizes"], ref["com"], L)
    edges = np.linspace(0.0, 1.0, 9)
    wts = np.linspace(-1.0, 1.0, 8)

    p = torch.from_numpy(pos).to("cuda:0").requires_grad_(True)
    mass, com, sigx, gid = fof_decorated(p, L, b, min_size=5)
    e = torch.from_numpy(edges).to(p.device)
    loss = (soft_histogram(sigx, e, 0.05) * torch.from_numpy(wts).to(p.device)).sum()
    loss.backward()
    np.testing.assert_allclose(sigx.detach().cpu().numpy(), sref, rtol=1e-9, atol=1e-12)

    s = torch.from_numpy(sref).requires_grad_(True)
    (soft_histogram(s, torch.from_numpy(edges), 0.05) * torch.from_numpy(wts)).sum().backward()
    want = oracle.dispersion_backward(pos, ref["group_id"], ref["sizes"], ref["com"], sref,
                                      s.grad.numpy(), L)
    got = p.grad.cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-5 * np.abs(want).max())
