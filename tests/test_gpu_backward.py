"""Frozen-assignment backward on the GPU (paper Sec. 3.1) against the FP64 oracle gradient
(1e-5 relative) and against central finite differences of the oracle's group statistics
with memberships held fixed (1e-3 relative)."""
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


def run_backward(pos, vel, L, b, min_size, seed):
    import torch
    from paper_2510_26851_amd.autograd import fof_stats

    dev = torch.device("cuda:0")
    p = torch.from_numpy(pos).to(dev).requires_grad_(True)
    v = torch.from_numpy(vel).to(dev).requires_grad_(True)
    mass, com, sigv, gid = fof_stats(p, v, L, b, min_size)
    G = mass.shape[0]
    rng = np.random.default_rng(seed)
    g_mass = torch.from_numpy(rng.standard_normal(G)).to(dev)
    g_com = torch.from_numpy(rng.standard_normal((G, 3))).to(dev)
    g_sig = torch.from_numpy(rng.standard_normal(G)).to(dev)
    J = (mass * g_mass).sum() + (com * g_com).sum() + (sigv * g_sig).sum()
    J.backward()
    torch.cuda.synchronize()
    return dict(G=G, gid=gid.cpu().numpy(), sizes=mass.detach().cpu().numpy().astype(np.int32),
                grad_pos=p.grad.cpu().numpy(), grad_vel=v.grad.cpu().numpy(),
                g_mass=g_mass.cpu().numpy(), g_com=g_com.cpu().numpy(), g_sig=g_sig.cpu().numpy(),
                com=com.detach().cpu().numpy(), sigv=sigv.detach().cpu().numpy())


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("which", ["clumpy", "config3"])
def test_frozen_backward_matches_fp64_oracle(which):
    if which == "clumpy":
        rng = np.random.default_rng(3)
        pos = W.clumpy_box(20000, 24.0, 10, 17)
        vel = rng.standard_normal(pos.shape).astype(np.float32)
        L, b, ms = 24.0, 0.35, 5
    else:
        box = W.config3()
        pos, vel, L, b, ms = box.pos, box.vel, box.L, box.b, box.min_size
    say(f"frozen backward {which} n={pos.shape[0]}")
    out = run_backward(pos, vel, L, b, ms, seed=5)
    root, _ = oracle.fof(pos, L, b)
    ref = oracle.groups(pos, root, L, ms, vel=vel)
    assert out["G"] == ref["n_groups"]
    np.testing.assert_array_equal(out["gid"], ref["group_id"])
    gp, gv = oracle.frozen_backward(ref["group_id"], ref["sizes"], ref["vmean"], ref["sigv"], vel,
                                    g_mass=out["g_mass"], g_com=out["g_com"], g_sigv=out["g_sig"])
    assert rel_err(out["grad_pos"], gp) <= 1e-5
    assert rel_err(out["grad_vel"], gv) <= 1e-5


def test_frozen_backward_matches_finite_differences():
    rng = np.random.default_rng(11)
    pos = W.clumpy_box(6000, 16.0, 5, 23)
    vel = rng.standard_normal(pos.shape).astype(np.float32)
    L, b, ms = 16.0, 0.4, 5
    say("frozen backward vs finite differences")
    out = run_backward(pos, vel, L, b, ms, seed=9)
    root, _ = oracle.fof(pos, L, b)

    def J(p, v):   # memberships frozen: the same root labels
        g = oracle.groups(p, root, L, ms, vel=v)
        return float((out["g_mass"] * g["sizes"]).sum() + (out["g_com"] * g["com"]).sum() +
                     (out["g_sig"] * g["sigv"]).sum())

    members = np.nonzero(out["gid"] >= 0)[0]
    scale = max(np.abs(out["grad_pos"]).max(), np.abs(out["grad_vel"]).max())
    for i in rng.choice(members, 8, replace=False):
        for a in range(3):
            for arr, grad in ((0, out["grad_pos"]), (1, out["grad_vel"])):
                h = 1e-3
                p1, v1, p2, v2 = pos.copy(), vel.copy(), pos.copy(), vel.copy()
                t1, t2 = (p1, p2) if arr == 0 else (v1, v2)
                t1[i, a] = np.float32(float(t1[i, a]) + h)
                t2[i, a] = np.float32(float(t2[i, a]) - h)
                den = float(t1[i, a]) - float(t2[i, a])
                fd = (J(p1, v1) - J(p2, v2)) / den
                assert abs(fd - grad[i, a]) <= 1e-3 * max(abs(grad[i, a]), 1e-2 * scale)


def test_forward_labels_unchanged_by_requires_grad():
    import torch
    from paper_2510_26851_amd import find_groups

    box = W.config0()
    say("forward identical with and without autograd")
    dev = torch.device("cuda:0")
    vel = np.random.default_rng(1).standard_normal(box.pos.shape).astype(np.float32)
    out = run_backward(box.pos, vel, box.L, box.b, box.min_size, seed=2)
    _, res = find_groups(torch.from_numpy(box.pos).to(dev), box.L, box.b, box.min_size)
    np.testing.assert_array_equal(out["gid"], res["group_id"].cpu().numpy())
