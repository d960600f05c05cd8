"""The Python binding refuses tensors the C ABI would misread (host memory, wrong element
type or size) before anything reaches the library: no GPU needed."""
import pytest
import torch

from paper_2510_26851_amd.fof import Plan


def fake_plan(n=8):
    plan = Plan.__new__(Plan)   # no device workspace: only the argument checks run
    plan.n = n
    plan.ws = torch.empty(0, dtype=torch.uint8, device="meta")
    plan.device = plan.ws.device
    return plan


def meta(shape, dtype):
    return torch.empty(shape, dtype=dtype, device="meta")


def test_build_grid_rejects_host_positions():
    with pytest.raises(ValueError, match="pos must be on"):
        fake_plan().build_grid(torch.zeros((8, 3)))


def test_subhalo_rejects_host_and_wrong_types():
    p, n = fake_plan(), 8
    good = dict(pos=meta((n, 3), torch.float32), vel=meta((n, 3), torch.float32),
                group_id=meta((n,), torch.int32), G=2, sizes=meta((2,), torch.int32),
                norm_x=None, norm_v=None, b6=1.0, sub=meta((n,), torch.int32))
    for key, bad, msg in (("pos", torch.zeros((n, 3)), "pos must be on"),
                          ("vel", meta((n, 3), torch.float64), "vel must be torch.float32"),
                          ("group_id", meta((n,), torch.int64), "group_id must be torch.int32"),
                          ("sizes", meta((1,), torch.int32), "sizes needs at least 2"),
                          ("sizes", meta((2,), torch.int64), "sizes must be torch.int32"),
                          ("sub", meta((n - 1,), torch.int32), "sub needs at least")):
        args = dict(good, **{key: bad})
        with pytest.raises(ValueError, match=msg):
            p.subhalo(**args)


def test_backward_and_dispersion_reject_host_tensors():
    p, n = fake_plan(), 8
    with pytest.raises(ValueError, match="group_id must be on"):
        p.backward(torch.zeros(n, dtype=torch.int32), 1, meta((1,), torch.int32))
    with pytest.raises(ValueError, match="g_com must be on"):
        p.backward(meta((n,), torch.int32), 1, meta((1,), torch.int32), g_com=torch.zeros((1, 3)))
    with pytest.raises(ValueError, match="grad_pos must be on"):
        p.backward_dispersion(meta((n, 3), torch.float32), meta((n,), torch.int32), 1,
                              meta((1,), torch.int32), meta((1, 3), torch.float64),
                              meta((1,), torch.float64), meta((1,), torch.float64),
                              torch.zeros((n, 3)))


def test_groups_refuses_reused_tables_of_another_shape():
    """Tables passed back in `out` must match the cap (by default the cap they came with)
    and the element types; otherwise the library would write past them."""
    p, n = fake_plan(), 8
    good = dict(group_id=meta((n,), torch.int32), n_groups=meta((1,), torch.int32),
                sizes=meta((4,), torch.int32), com=meta((4, 3), torch.float64), cap=4)
    for key, bad, msg in (("sizes", meta((3,), torch.int32), "sizes must have shape"),
                          ("com", meta((4, 3), torch.float32), "com must be torch.float64"),
                          ("group_id", torch.zeros(n, dtype=torch.int32), "group_id must be on"),
                          ("n_groups", meta((2,), torch.int32), "n_groups must have shape")):
        with pytest.raises(ValueError, match=msg):
            p.groups(20, out=dict(good, **{key: bad}))
    with pytest.raises(ValueError, match="sizes must have shape"):
        p.groups(20, cap=5, out=good)
