"""Helpers shared by the GPU tests: run the HIP path through the C ABI and compare it with
the CPU oracle."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(pos, L, b, min_size, vel=None, tune=None, cap=None):
    import torch
    from paper_2510_26851_amd import Plan, trim

    n = pos.shape[0]
    dev = torch.device("cuda:0")
    t = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    v = None if vel is None else torch.from_numpy(np.ascontiguousarray(vel)).to(dev)
    plan = Plan([n], [(L, b)], device=dev, tune=tune)
    plan.build_grid(t)
    root = plan.link()
    res = trim(plan.groups(min_size, vel=v, cap=cap))
    torch.cuda.synchronize()
    out = {k: (val.cpu().numpy() if hasattr(val, "cpu") else val) for k, val in res.items()}
    return root.cpu().numpy(), out, plan.status()


def com_close(got, ref, L, spacing, rtol=1e-5):
    """C28 reading: |minimum-image(com - ref)| / max(|ref|, mean spacing) <= rtol per axis."""
    L = np.broadcast_to(np.asarray(L, np.float64), (3,))
    d = got - ref
    d = d - L * np.round(d / L)
    scale = np.maximum(np.abs(ref), spacing)
    return np.all(np.abs(d) <= rtol * scale)


def compare_with_oracle(pos, L, b, min_size, vel=None, tune=None, cap=None, root_ref=None):
    root, g, status = run_gpu(pos, L, b, min_size, vel=vel, tune=tune, cap=cap)
    assert status == 0, f"status word {status}"
    if root_ref is None:
        root_ref, _ = oracle.fof(pos, L, b)
    np.testing.assert_array_equal(root, root_ref)
    ref = oracle.groups(pos, root_ref, L, min_size, vel=vel, cap=cap)
    assert g["n_groups"] == ref["n_groups"]
    np.testing.assert_array_equal(g["group_id"], ref["group_id"])
    np.testing.assert_array_equal(g["sizes"], ref["sizes"])
    n = pos.shape[0]
    Lv = np.broadcast_to(np.asarray(L, np.float64), (3,))
    spacing = (np.prod(Lv) / max(n, 1)) ** (1.0 / 3.0)
    assert com_close(g["com"], ref["com"], L, spacing)
    if vel is not None:
        np.testing.assert_allclose(g["vmean"], ref["vmean"], rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(g["sigv"], ref["sigv"], rtol=1e-5, atol=1e-9)
    return root, g
