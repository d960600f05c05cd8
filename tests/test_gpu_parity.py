"""Parity of the HIP path (through the C ABI) with the CPU oracle on the same seeded inputs.

Labels, group ids and sizes must match bit-exactly; centres of mass, mean velocities and
dispersions within 1e-5 relative (minimum-image difference over max(|ref|, mean spacing)).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import compare_with_oracle, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_26851_amd  # noqa: F401  (raises if libfof.so is missing)


@pytest.mark.parametrize("seed,n,L,b", [
    (1, 1, 10.0, 0.6),
    (2, 2, 1.0, 0.45),
    (3, 63, 3.0, 0.6),
    (4, 65, 3.0, 0.6),
    (5, 1000, 10.0, 0.6),
    (6, 4097, 16.0, 0.9),
    (7, 3000, (12.0, 9.0, 20.0), 0.7),
    (8, 800, 3.0, 0.35),
    (9, 200, 1.0, 0.4),          # 2 coarse cells per axis
    (10, 50, (0.7, 3.0, 5.0), 0.34),
    (11, 20000, 20.0, 0.5),
])
def test_uniform_boxes(seed, n, L, b):
    say(f"uniform seed={seed} n={n} L={L} b={b}")
    pos = W.uniform_box(n, np.broadcast_to(L, (3,)), seed)
    compare_with_oracle(pos, L, b, min_size=2)


@pytest.mark.parametrize("seed,n,L,ncl,b", [
    (21, 5000, 24.0, 6, 0.5),
    (22, 30000, 40.0, 20, 0.4),
    (23, 12000, 8.0, 3, 0.3),
])
def test_clumpy_boxes(seed, n, L, ncl, b):
    say(f"clumpy seed={seed} n={n}")
    pos = W.clumpy_box(n, L, ncl, seed)
    compare_with_oracle(pos, L, b, min_size=5)


def test_empty_box():
    say("empty box")
    root, g, status = run_gpu(np.zeros((0, 3), np.float32), 10.0, 0.5, 2)
    assert root.shape == (0,) and g["n_groups"] == 0 and status == 0


def test_lattice_closed_cases():
    say("lattice one group")
    pos = W.cubic_lattice(24, 0.375)             # spacing < b: one group of 13824
    root, g, _ = run_gpu(pos, 9.0, 0.4, 20)
    assert np.all(root == 0) and g["n_groups"] == 1 and g["sizes"][0] == 24 ** 3
    say("lattice singletons")
    pos = W.cubic_lattice(24, 0.4375)            # spacing > b: all singletons
    root, g, _ = run_gpu(pos, 10.5, 0.4, 1)
    np.testing.assert_array_equal(root, np.arange(24 ** 3))
    assert g["n_groups"] == 24 ** 3
    np.testing.assert_array_equal(g["group_id"], np.arange(24 ** 3))


def test_min_size_one_and_cap_overflow():
    say("min_size 1 + cap overflow")
    pos = W.clumpy_box(3000, 12.0, 4, 31)
    root_ref, _ = oracle.fof(pos, 12.0, 0.45)
    ref = oracle.groups(pos, root_ref, 12.0, 1)
    root, g, _ = run_gpu(pos, 12.0, 0.45, 1)
    np.testing.assert_array_equal(root, root_ref)
    assert g["n_groups"] == ref["n_groups"]
    np.testing.assert_array_equal(g["group_id"], ref["group_id"])
    np.testing.assert_array_equal(g["sizes"], ref["sizes"])
    cap = 17
    root, g, _ = run_gpu(pos, 12.0, 0.45, 1, cap=cap)
    assert g["n_groups"] == ref["n_groups"] and g["sizes"].shape[0] == cap
    np.testing.assert_array_equal(g["sizes"], ref["sizes"][:cap])


def test_out_of_range_sets_status():
    say("status word: out-of-range and NaN inputs")
    pos = W.uniform_box(500, (10.0,) * 3, 3)
    pos[7, 1] = 10.0          # x == L is outside [0, L)
    pos[11, 2] = np.nan
    _, _, status = run_gpu(pos, 10.0, 0.5, 2)
    assert status & 1


@pytest.mark.parametrize("tune", [dict(block=64), dict(block=128), dict(block=512),
                                  dict(block=1024), dict(cell_side=0.5), dict(cell_side=3.0),
                                  dict(flags=1)])
def test_launch_shape_and_cell_side_do_not_change_results(tune):
    say(f"launch shape {tune}")
    box = W.config0()
    root_ref, _ = oracle.fof(box.pos, box.L, box.b)
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, tune=tune, root_ref=root_ref)


def test_config0_clumps_32768():
    box = W.config0()
    say(f"config0 {box.name}")
    root, g = compare_with_oracle(box.pos, box.L, box.b, box.min_size)
    assert g["n_groups"] > 10


def test_config3_zeldovich_128_with_velocities():
    box = W.config3()
    say(f"config3 {box.name} n={box.n}")
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, vel=box.vel)


def test_repeat_runs_identical():
    box = W.config3()
    say("repeat runs")
    r1, g1, _ = run_gpu(box.pos, box.L, box.b, box.min_size)
    r2, g2, _ = run_gpu(box.pos, box.L, box.b, box.min_size)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(g1["group_id"], g2["group_id"])


def very_dense_box(seed=41):
    """20000 uniform particles plus 4 clumps of 10000 with sigma 0.12 in L = 24: several
    coarse cells hold more than 2048 particles (the staging path of the clique sort)."""
    rng = np.random.default_rng(seed)
    L = 24.0
    uni = rng.random((20000, 3)) * L
    centres = rng.random((4, 3)) * L
    mem = np.concatenate([c + 0.12 * rng.standard_normal((10000, 3)) for c in centres])
    pos = W.wrap_to_f32(np.concatenate([uni, mem]), (L, L, L))
    b = W.linking_length(0.2, L, pos.shape[0])
    return pos, L, b


@pytest.mark.parametrize("thr", [1, 4, 8, 32, 200, -1])
def test_dense_threshold_does_not_change_results(thr):
    say(f"dense threshold {thr}")
    box = W.config0()
    root_ref, _ = oracle.fof(box.pos, box.L, box.b)
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, tune=dict(dense_threshold=thr),
                        root_ref=root_ref)


@pytest.mark.parametrize("thr", [0, 1, 16, -1])
def test_very_dense_clumps(thr):
    pos, L, b = very_dense_box()
    say(f"very dense clumps thr={thr} n={pos.shape[0]} b={b}")
    compare_with_oracle(pos, L, b, 20, tune=dict(dense_threshold=thr))


@pytest.mark.parametrize("cell_side", [0.0, 1.0, 2.5])
def test_very_dense_clumps_cell_side(cell_side):
    pos, L, b = very_dense_box(43)
    say(f"very dense clumps cell_side={cell_side}")
    compare_with_oracle(pos, L, b, 20, tune=dict(cell_side=cell_side))


def test_autotuner_choice_does_not_change_results(tmp_path):
    import torch
    from paper_2510_26851_amd.tune import autotune

    box = W.config0()
    say("autotuner on config 0")
    pos = torch.from_numpy(box.pos).cuda()
    tune = autotune(pos, box.L, box.b, box.min_size, cache=str(tmp_path / "tune.json"), reps=1)
    assert autotune(pos, box.L, box.b, box.min_size, cache=str(tmp_path / "tune.json")) == tune
    root_ref, _ = oracle.fof(box.pos, box.L, box.b)
    compare_with_oracle(box.pos, box.L, box.b, box.min_size, tune=tune, root_ref=root_ref)


@pytest.mark.parametrize("tune", [
    dict(dense_threshold=-1, cell_side=0.68),   # halos over the LDS cap, z-windows that fit
    dict(dense_threshold=-1, cell_side=2.0),    # single z-layers too full: global search
    dict(link_edges=1),                         # deferred hooks overflow: tiles relinked
    dict(link_edges=1, dense_threshold=8),
])
def test_overflow_paths_of_the_tiled_link(tune):
    say(f"overflow paths {tune}")
    pos = W.clumpy_box(100000, 20.0, 30, 41)
    compare_with_oracle(pos, 20.0, 0.3, 5, tune=tune)


def test_grid_over_2_27_cells_takes_the_two_level_binning():
    """A grid of more than 2^27 cells (16384 sorting buckets of 8192 cells) is binned in two
    levels: placed by buckets of 2^16 cells, then each split into its sorting buckets (the
    path a 1024^3 box takes).  Every label, group id, size and centre of mass of the
    17M-particle box against the oracle run on the whole box, for that grid and for the
    default one (one level)."""
    import torch
    from paper_2510_26851_amd import Plan, trim

    from gpu_util import com_close

    n, L = 17_000_000, 256.0
    b = W.linking_length(0.2, L, n)
    pos = W.clumpy_box(n, L, 4000, 51)
    say(f"two-level binning: oracle on n={n}")
    ref_root, _ = oracle.fof_par(pos, L, b)
    ref = oracle.groups(pos, ref_root, L, 20)
    assert ref["n_groups"] > 0
    t = torch.from_numpy(pos).to("cuda:0")
    for side, over in [(0.25, True), (0.0, False)]:
        say(f"two-level binning check: n={n} cell_side={side}")
        plan = Plan([n], [(L, b)], device=t.device, tune=dict(cell_side=side))
        assert (plan.grid.ncell > (1 << 27)) == over, plan.grid.ncell
        plan.build_grid(t)
        root = plan.link()
        res = trim(plan.groups(20))
        torch.cuda.synchronize()
        assert plan.status() == 0
        np.testing.assert_array_equal(root.cpu().numpy(), ref_root)
        assert res["n_groups"] == ref["n_groups"]
        np.testing.assert_array_equal(res["group_id"].cpu().numpy(), ref["group_id"])
        np.testing.assert_array_equal(res["sizes"].cpu().numpy(), ref["sizes"])
        assert com_close(res["com"].cpu().numpy(), ref["com"], L, L / n ** (1 / 3))
        del plan, root, res


def test_few_particles_on_a_huge_grid_take_the_per_particle_binning():
    """200k particles with b = 0.05 in a box of side 256: clique cells of side < b / sqrt(3)
    force 890^3 coarse cells, and 7 placing blocks are too few to split 16384 buckets into
    8 sorting buckets each, so the binning takes one rank atomic per particle.  Labels and
    groups against the oracle."""
    import torch
    from paper_2510_26851_amd import Plan, trim

    n, L, b = 200_000, 256.0, 0.05
    pos = W.clumpy_box(n, L, 300, 53)
    say(f"per-particle binning: n={n} b={b}")
    ref_root, _ = oracle.fof_par(pos, L, b)
    ref = oracle.groups(pos, ref_root, L, 2)
    t = torch.from_numpy(pos).to("cuda:0")
    plan = Plan([n], [(L, b)], device=t.device)
    assert plan.grid.ncell > 1 << 29, plan.grid.ncell
    plan.build_grid(t)
    root = plan.link()
    res = trim(plan.groups(2))
    torch.cuda.synchronize()
    assert plan.status() == 0
    np.testing.assert_array_equal(root.cpu().numpy(), ref_root)
    assert res["n_groups"] == ref["n_groups"] > 0
    np.testing.assert_array_equal(res["group_id"].cpu().numpy(), ref["group_id"])
    np.testing.assert_array_equal(res["sizes"].cpu().numpy(), ref["sizes"])
    del plan, root, res


@pytest.mark.parametrize("n", [5000, 40000])
def test_all_particles_at_one_point(n):
    """Degenerate input: one cell holds every particle (the bucketed binning then sorts one
    bucket larger than a block's register chunk, and the dense path stages through HBM).
    Closed form: one group of n, labelled 0, centred on the point."""
    say(f"all {n} particles at one point")
    pos = np.full((n, 3), 3.3, np.float32)
    root, g, status = run_gpu(pos, 10.0, 0.5, 2)
    assert status == 0
    assert np.all(root == 0) and g["n_groups"] == 1 and g["sizes"][0] == n
    np.testing.assert_array_equal(g["com"][0], np.float64(np.float32(3.3)) * np.ones(3))


def test_two_points_and_the_box_edge():
    """Two points of 20000 particles each, and pairs straddling the periodic edge: one at
    0.0, one at the largest float32 below L (closer than b through the boundary)."""
    say("two points + edge pairs")
    L = 10.0
    below = np.nextafter(np.float32(L), np.float32(0))
    a = np.full((20000, 3), 2.0, np.float32)
    b_ = np.full((20000, 3), 7.0, np.float32)
    edge = np.array([[0.0, 5.0, 5.0], [below, 5.0, 5.0],
                     [5.0, 0.0, 1.0], [5.0, below, 1.0]], np.float32)
    pos = np.concatenate([a, b_, edge])
    root, g, status = run_gpu(pos, L, 0.5, 2)
    assert status == 0
    assert np.all(root[:20000] == 0) and np.all(root[20000:40000] == 20000)
    np.testing.assert_array_equal(root[40000:], [40000, 40000, 40002, 40002])
    assert g["n_groups"] == 4
    np.testing.assert_array_equal(g["sizes"], [20000, 20000, 2, 2])
    # the edge pairs' centres sit on the boundary (wrapped into [0, L))
    c = g["com"][2]
    assert min(c[0], L - c[0]) < 1e-5 and abs(c[1] - 5.0) < 1e-6 and abs(c[2] - 5.0) < 1e-6


def test_dense_cells_beyond_the_table_cap_take_the_plain_path():
    """With clique tables for only a few dense cells, the others are linked as ordinary
    cells (tiles, z-windows, global search) and the status word says so: labels, groups
    and centres still equal the oracle's."""
    pos = W.clumpy_box(60000, 24.0, 14, 4242)
    L, b = 24.0, 0.35
    say("dense table cap: 6 tables")
    for tune in (dict(dense_cells=6), dict(dense_cells=6, dense_threshold=16)):
        root, g, status = run_gpu(pos, L, b, 20, tune=tune)
        assert status == 2, status   # FOF_STATUS_DENSE_CAP
        ref_root, _ = oracle.fof(pos, L, b)
        np.testing.assert_array_equal(root, ref_root)
        ref = oracle.groups(pos, ref_root, L, 20)
        assert g["n_groups"] == ref["n_groups"]
        np.testing.assert_array_equal(g["sizes"], ref["sizes"])
        np.testing.assert_array_equal(g["group_id"], ref["group_id"])
