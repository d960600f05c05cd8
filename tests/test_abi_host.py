"""Host-only checks of libfof.so: it loads, exports every symbol include/fof.h declares, and
rejects bad arguments on the host before anything would be enqueued (no GPU needed)."""
import ctypes
import math
import os
import re
import struct

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fof.h")

_lib = pytest.importorskip("paper_2510_26851_amd._lib")


def lib():
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fof_[a-z_]+)\s*\(", text)))


def test_header_declarations_are_exported():
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    L = lib()
    for f in names:
        assert hasattr(L, f), f


def test_strerror():
    assert _lib.strerror(0) == "ok"
    assert "invalid" in _lib.strerror(-1)
    assert _lib.strerror(12345) == "unknown error"


def plan(counts, boxes, tune=None, desc=True):
    nbox = len(counts)
    c = np.asarray(counts, dtype=np.int64)
    bx = (_lib.fof_box * nbox)()
    for k, (L, b) in enumerate(boxes):
        L3 = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
        bx[k].L[:] = [float(v) for v in L3]
        bx[k].b = b
    g = _lib.fof_grid()
    t = ctypes.byref(tune) if tune is not None else None
    rc = lib().fof_workspace_bytes(nbox, c.ctypes.data_as(ctypes.c_void_p), bx, t, ctypes.byref(g),
                                   None, 0)
    if rc or not desc:
        return rc, g, None
    buf = np.zeros(g.desc_bytes, np.uint8)
    rc = lib().fof_workspace_bytes(nbox, c.ctypes.data_as(ctypes.c_void_p), bx, t,
                                   ctypes.byref(g), buf.ctypes.data_as(ctypes.c_void_p),
                                   buf.shape[0])
    return rc, g, buf


# BoxDesc layout (fof_internal.h): int64 off, cell_base, tile_base; int32 n, m, nc[3], nf[3],
# R, dense_ok, tiled, ntile[3]; double L[3], halfL[3], b2; float inv_fine[3], side[3],
# reach, fine_side, fine[3], slack.
_DESC = struct.Struct("<qqqii3i3iiii3i3d3dd3f3fff3ff3f")


def desc_stride():
    rc, g, _ = plan([1], [(10.0, 0.5)], desc=False)
    return g.desc_bytes


def decode(buf, k=0):
    v = _DESC.unpack_from(buf.tobytes(), k * desc_stride())
    return dict(off=v[0], cell_base=v[1], tile_base=v[2], n=v[3], m=v[4], nc=v[5:8],
                nf=v[8:11], R=v[11], dense_ok=v[12], tiled=v[13], ntile=v[14:17], L=v[17:20],
                halfL=v[20:23], b2=v[23], inv_fine=v[24:27], side=v[27:30], reach=v[30],
                fine_side=v[31], fine=v[32:35], slack=v[35], Lup=v[36:39])


@pytest.mark.parametrize("L", [512.0, 64.0, 0.7, 50.397, 1.0 / 3.0, 123456.789])
def test_float_bound_of_the_box_length(L):
    """Lup is the smallest float >= L, so the binning's float test x < Lup accepts exactly
    the floats x with x < L in exact arithmetic."""
    rc, g, buf = plan([10], [(L, L / 8)])
    assert rc == 0
    up = np.float32(decode(buf)["Lup"][0])
    assert float(up) >= L and float(np.nextafter(up, np.float32(0))) < L


def test_descriptor_size():
    rc, g, buf = plan([10, 20], [(10.0, 0.5), (10.0, 0.5)])
    st = desc_stride()
    assert rc == 0 and g.desc_bytes == 2 * st and _DESC.size <= st and st % 16 == 0


@pytest.mark.parametrize("L,b,n", [(64.0, 0.4, 32768), (512.0, 0.2, 512 ** 3), (256.0, 0.2, 256 ** 3),
                                   (1.0, 0.4, 50), (0.9, 0.44, 100), ((0.7, 3.0, 5.0), 0.34, 50),
                                   (50.397, 0.4, 16000)])
def test_plan_geometry_guarantees(L, b, n):
    """Coarse cells are at least b plus twice the float32 index error, so the 27-cell stencil
    is complete; fine cells are cliques (any two members closer than 0.999 b)."""
    rc, g, buf = plan([n], [(L, b)])
    assert rc == 0
    d = decode(buf)
    L3 = np.broadcast_to(np.asarray(L, np.float64), (3,))
    Lmax = float(L3.max())
    eps = Lmax * 2.0 ** -23 * (1 + 2.0 ** -10)
    for a in range(3):
        side = L3[a] / d["nc"][a]
        assert d["nc"][a] == 1 or side >= b + 2 * eps
        fine = side / d["m"]
        assert d["nf"][a] == d["nc"][a] * d["m"]
        assert float(np.float32(d["inv_fine"][a])) == float(np.float32(d["nf"][a] / L3[a]))
    fine_max = max(L3[a] / d["nc"][a] / d["m"] for a in range(3))
    assert math.sqrt(3.0) * (fine_max + 2 * eps) <= 0.999 * b * (1 + 1e-12)
    assert d["reach"] >= b + 2.5 * Lmax * 2.0 ** -23
    assert d["b2"] == b * b
    # a friend's fine cell is at most R away per axis; fine_side is a lower bound
    a_min = min(L3[a] / d["nf"][a] for a in range(3))
    assert d["R"] * a_min >= b + 2 * eps
    assert d["fine_side"] <= a_min - 2 * eps
    assert d["dense_ok"] == int(min(d["nc"]) >= 3 and d["R"] <= 3)
    assert d["slack"] >= 4 * eps
    ncell = int(np.prod(d["nc"]))
    assert g.ncell == ncell and ncell <= 8 * n + 64 + 3 * max(d["nc"]) ** 2 * 3
    assert g.ws_bytes > 0 and g.ws_bytes % 256 == 0


def test_batch_plan_offsets():
    counts = [100, 0, 57, 1000]
    boxes = [(10.0, 0.4), (5.0, 0.3), (8.0, 0.5), (20.0, 0.4)]
    rc, g, buf = plan(counts, boxes)
    assert rc == 0 and g.nbox == 4 and g.n == sum(counts)
    off, cb = 0, 0
    for k in range(4):
        d = decode(buf, k)
        assert d["off"] == off and d["cell_base"] == cb and d["n"] == counts[k]
        off += counts[k]
        cb += int(np.prod(d["nc"]))
    assert g.ncell == cb


@pytest.mark.parametrize("counts,boxes", [
    ([10], [(10.0, 0.0)]),           # b = 0
    ([10], [(10.0, -1.0)]),          # b < 0
    ([10], [(1.0, 0.5)]),            # 2b == L
    ([10], [(0.0, 0.1)]),            # L = 0
    ([10], [(float("inf"), 0.1)]),   # L not finite
    ([10], [(10.0, float("nan"))]),  # b NaN
    ([-1], [(10.0, 0.4)]),           # negative count
    ([2 ** 31], [(4096.0, 0.4)]),    # total above INT32_MAX
])
def test_plan_rejects_bad_arguments(counts, boxes):
    rc, _, _ = plan(counts, boxes, desc=False)
    assert rc == _lib.FOF_EINVAL


def test_plan_rejects_bad_tune():
    t = _lib.fof_tune()
    t.block = 100     # not a multiple of 64
    rc, _, _ = plan([10], [(10.0, 0.4)], tune=t, desc=False)
    assert rc == _lib.FOF_EINVAL
    t = _lib.fof_tune()
    t.flags = 2       # unknown flag bit
    rc, _, _ = plan([10], [(10.0, 0.4)], tune=t, desc=False)
    assert rc == _lib.FOF_EINVAL
    t = _lib.fof_tune()
    t.link_edges = -1
    rc, _, _ = plan([10], [(10.0, 0.4)], tune=t, desc=False)
    assert rc == _lib.FOF_EINVAL
    t = _lib.fof_tune()
    t.dense_cells = -1
    rc, _, _ = plan([10], [(10.0, 0.4)], tune=t, desc=False)
    assert rc == _lib.FOF_EINVAL


def test_dense_table_cap_follows_the_tune():
    """The clique tables are sized for n / (threshold + 1) dense cells, or for the tune's
    dense_cells when that is smaller (the rest take the plain path on the device)."""
    t = _lib.fof_tune()
    rc, g0, _ = plan([40000], [(40.0, 0.4)], tune=t, desc=False)
    assert rc == 0 and g0.dense_cap == 40000 // (g0.dense_threshold + 1) + 1
    t.dense_cells = 7
    rc, g1, _ = plan([40000], [(40.0, 0.4)], tune=t, desc=False)
    assert rc == 0 and g1.dense_cap == 7 and g1.ws_bytes < g0.ws_bytes
    t.dense_cells = 10 ** 9
    rc, g2, _ = plan([40000], [(40.0, 0.4)], tune=t, desc=False)
    assert rc == 0 and g2.dense_cap == g0.dense_cap


def test_link_edge_capacity_sets_the_workspace():
    t = _lib.fof_tune()
    rc, g0, _ = plan([40000], [(40.0, 0.4)], tune=t, desc=False)
    assert rc == 0 and g0.link_edges == 40000 // 4 + 65536
    t.link_edges = 5
    rc, g1, _ = plan([40000], [(40.0, 0.4)], tune=t, desc=False)
    assert rc == 0 and g1.link_edges == 5 and g1.ws_bytes < g0.ws_bytes


def test_no_tiles_flag_clears_the_tiled_bit():
    t = _lib.fof_tune()
    rc, g, buf = plan([4000], [(40.0, 0.4)], tune=t)
    assert rc == 0 and decode(buf, 0)["tiled"] == 1 and g.ntiles > 0
    t.flags = _lib.FOF_TUNE_NO_TILES
    rc, g, buf = plan([4000], [(40.0, 0.4)], tune=t)
    assert rc == 0 and decode(buf, 0)["tiled"] == 0 and g.ntiles == 0


def test_plan_rejects_small_desc_buffer():
    c = np.array([10], np.int64)
    bx = (_lib.fof_box * 1)()
    bx[0].L[:] = [10.0, 10.0, 10.0]
    bx[0].b = 0.4
    g = _lib.fof_grid()
    buf = np.zeros(16, np.uint8)
    rc = lib().fof_workspace_bytes(1, c.ctypes.data_as(ctypes.c_void_p), bx, None, ctypes.byref(g),
                                   buf.ctypes.data_as(ctypes.c_void_p), 16)
    assert rc == _lib.FOF_EINVAL


def test_entry_points_reject_bad_arguments_before_launch():
    L = lib()
    rc, g, _ = plan([100], [(10.0, 0.4)])
    assert rc == 0
    gp = ctypes.byref(g)
    fake_ws = ctypes.c_void_p(0x100000)      # never dereferenced: every call below fails first
    misaligned = ctypes.c_void_p(0x100010)
    W = g.ws_bytes
    assert L.fof_build_grid(None, None, fake_ws, W, None) == _lib.FOF_EINVAL
    assert L.fof_build_grid(gp, None, fake_ws, W, None) == _lib.FOF_EINVAL       # pos NULL
    assert L.fof_build_grid(gp, fake_ws, misaligned, W, None) == _lib.FOF_EINVAL  # alignment
    assert L.fof_build_grid(gp, fake_ws, None, W, None) == _lib.FOF_EINVAL       # ws NULL
    assert L.fof_link(gp, fake_ws, W, None, None, None) == _lib.FOF_EINVAL       # root NULL
    S = _lib.fof_sample()                                                        # K = 0
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.K, S.tau, S.b, S.edge_cap = 4, 0.01, 0.2, 100
    S.n_edges, S.ei, S.ej, S.d2 = 0x100000, 0x100000, 0x100000, 0x100000
    S.scratch, S.scratch_bytes = 0x100000, 10                                   # too small
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.scratch_bytes = _lib.sample_scratch_bytes(100, 4, 100)
    S.tau = 0.0                                                                  # tau <= 0
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.tau, S.K = 0.01, 65536                                                     # K too large
    S.scratch_bytes = _lib.sample_scratch_bytes(100, 65536, 100)
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.K, S.tau = 4, 0.01
    S.scratch_bytes = _lib.sample_scratch_bytes(100, 4, 100)
    S.s_first = -1                                                               # s_first < 0
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.s_first = 2 ** 31 - 4                                                      # past 2^31 - 1
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.s_first = 0
    S.form, S.alpha = _lib.FOF_PROB_QUADRATIC, 0.0                              # alpha <= 0
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.form, S.alpha = 2, 1.0                                                     # unknown form
    assert L.fof_link(gp, fake_ws, W, ctypes.byref(S), fake_ws, None) == _lib.FOF_EINVAL
    S.form = _lib.FOF_PROB_DISTANCE
    # the sampled catalogue: min_size >= 2, no per-particle or velocity outputs
    Sp = ctypes.byref(S)
    assert L.fof_groups(gp, fake_ws, W, Sp, 1, None, 10, None, fake_ws, fake_ws, fake_ws, None,
                        None, None) == _lib.FOF_EINVAL                            # min_size 1
    assert L.fof_groups(gp, fake_ws, W, Sp, 2, fake_ws, 10, None, fake_ws, fake_ws, fake_ws,
                        None, None, None) == _lib.FOF_EINVAL                      # vel given
    assert L.fof_groups(gp, fake_ws, W, Sp, 2, None, 10, fake_ws, fake_ws, fake_ws, fake_ws,
                        None, None, None) == _lib.FOF_EINVAL                      # group_id
    assert L.fof_groups(gp, fake_ws, W, Sp, 2, None, 10, None, fake_ws, fake_ws, None, None,
                        None, None) == _lib.FOF_EINVAL                            # com NULL
    S.tau = 0.0
    assert L.fof_groups(gp, fake_ws, W, Sp, 2, None, 10, None, fake_ws, fake_ws, fake_ws, None,
                        None, None) == _lib.FOF_EINVAL                            # bad sample
    assert L.fof_group_dispersion(gp, fake_ws, W, -1, fake_ws, fake_ws, fake_ws, fake_ws,
                                  None) == _lib.FOF_EINVAL                        # cap < 0
    assert L.fof_group_dispersion(gp, fake_ws, W, 10, None, fake_ws, fake_ws, fake_ws,
                                  None) == _lib.FOF_EINVAL                        # n_groups NULL
    assert L.fof_group_dispersion(gp, fake_ws, W, 10, fake_ws, fake_ws, None, fake_ws,
                                  None) == _lib.FOF_EINVAL                        # com NULL
    assert L.fof_backward_dispersion(gp, fake_ws, W, fake_ws, fake_ws, -1, fake_ws, fake_ws,
                                     fake_ws, fake_ws, fake_ws, None) == _lib.FOF_EINVAL  # G < 0
    assert L.fof_backward_dispersion(gp, fake_ws, W, None, fake_ws, 3, fake_ws, fake_ws,
                                     fake_ws, fake_ws, fake_ws, None) == _lib.FOF_EINVAL
    assert L.fof_groups(gp, fake_ws, W, None, 20, None, 10, None, fake_ws, fake_ws, None, None,
                        None, None) == _lib.FOF_EINVAL                            # group_id NULL
    assert L.fof_groups(gp, fake_ws, W, None, 20, None, -1, fake_ws, fake_ws, fake_ws, None,
                        None, None, None) == _lib.FOF_EINVAL                      # cap < 0
    assert L.fof_groups(gp, fake_ws, W, None, 20, None, 10, fake_ws, fake_ws, None, None, None,
                        None, None) == _lib.FOF_EINVAL                            # sizes NULL
    assert L.fof_groups(gp, fake_ws, W, None, 20, fake_ws, 10, fake_ws, fake_ws, fake_ws, None,
                        fake_ws, None, None) == _lib.FOF_EINVAL                   # vmean w/o sigv
    F = _lib.FOF_FROZEN
    nul = [None] * 3
    assert L.fof_backward(gp, fake_ws, W, F, None, 1, fake_ws, *nul, None, None, None, None,
                          None, 0, None, None, None) == _lib.FOF_EINVAL          # group_id NULL
    assert L.fof_backward(gp, fake_ws, W, F, fake_ws, -1, fake_ws, *nul, None, None, None, None,
                          None, 0, None, None, None) == _lib.FOF_EINVAL          # G < 0
    assert L.fof_backward(gp, fake_ws, W, F, fake_ws, 1, fake_ws, *nul, None, None, fake_ws,
                          None, None, 0, None, fake_ws, None) == _lib.FOF_EINVAL  # vel missing
    assert L.fof_backward(gp, fake_ws, W, 7, fake_ws, 1, fake_ws, *nul, None, None, None, None,
                          None, 0, None, None, None) == _lib.FOF_EINVAL          # bad mode
    assert L.fof_backward(gp, fake_ws, W, _lib.FOF_SCORE, None, 0, None, *nul, None, None, None,
                          None, fake_ws, 2, fake_ws, None, None) == _lib.FOF_EINVAL  # no sample
    need = L.fof_subhalo_scratch_bytes(100, 3)
    assert need >= 12 * 100 + 4 * 2 * 3
    sub_args = [fake_ws, fake_ws, fake_ws, 3, fake_ws, fake_ws, fake_ws, 1.0, fake_ws, need,
                fake_ws, None]

    def subhalo(ws_bytes=W, **kw):
        a = list(sub_args)
        names = ["pos", "vel", "gid", "G", "sizes", "nx", "nv", "b6", "scratch", "nbytes", "sub",
                 "stream"]
        for k, v in kw.items():
            a[names.index(k)] = v
        return L.fof_subhalo(gp, fake_ws, ws_bytes, *a)

    assert subhalo(b6=0.0) == _lib.FOF_EINVAL                                    # b6 <= 0
    assert subhalo(b6=float("nan")) == _lib.FOF_EINVAL                           # b6 not finite
    assert subhalo(G=-1) == _lib.FOF_EINVAL                                      # G < 0
    assert subhalo(G=101) == _lib.FOF_EINVAL                                     # G > n
    assert subhalo(sub=None) == _lib.FOF_EINVAL                                  # sub NULL
    assert subhalo(vel=None) == _lib.FOF_EINVAL                                  # vel NULL
    assert subhalo(nbytes=need - 1) == _lib.FOF_EINVAL                           # scratch small
    assert subhalo(scratch=misaligned) == _lib.FOF_EINVAL                        # alignment
    assert subhalo(ws_bytes=W - 1) == _lib.FOF_ENOMEM                            # ws small
    p = ctypes.c_void_p()
    assert L.fof_status(gp, misaligned, W, ctypes.byref(p)) == _lib.FOF_EINVAL
    assert L.fof_status(gp, fake_ws, W, ctypes.byref(p)) == 0
    assert p.value == 0x100000 + g.off_status


def test_every_workspace_call_reports_a_small_workspace():
    """FOF_ENOMEM: the workspace the caller passes is smaller than the plan needs; nothing is
    enqueued (the fake workspace is never touched)."""
    L = lib()
    rc, g, _ = plan([100], [(10.0, 0.4)])
    assert rc == 0
    gp = ctypes.byref(g)
    ws = ctypes.c_void_p(0x100000)
    small = g.ws_bytes - 256
    E = _lib.FOF_ENOMEM
    p = ctypes.c_void_p()
    assert L.fof_build_grid(gp, ws, ws, small, None) == E
    assert L.fof_link(gp, ws, small, None, ws, None) == E
    assert L.fof_groups(gp, ws, small, None, 20, None, 10, ws, ws, ws, ws, None, None, None) == E
    assert L.fof_group_dispersion(gp, ws, small, 10, ws, ws, ws, ws, None) == E
    assert L.fof_backward_dispersion(gp, ws, small, ws, ws, 1, ws, ws, ws, ws, ws, None) == E
    assert L.fof_backward(gp, ws, small, _lib.FOF_SCORE, None, 0, None, None, None, None, None,
                          None, None, None, ws, 2, ws, None, None) == E
    assert L.fof_status(gp, ws, small, ctypes.byref(p)) == E
    assert L.fof_status(gp, ws, 0, ctypes.byref(p)) == E
    assert L.fof_strerror(E) == b"workspace too small"


def test_one_hip_runtime_per_process():
    """Loading the library (even before anything imports torch) must leave one HIP runtime
    mapped: two copies in one process give 'no device' on the second."""
    import subprocess
    import sys

    code = ("import paper_2510_26851_amd, torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"


def test_plan_counts_the_particles_of_boxes_without_tiles():
    # a 3-wide box is too small for link tiles (it needs 18 cells along z), a 40-wide one is
    rc, g, buf = plan([100, 40000], [(3.0, 0.4), (40.0, 0.4)])
    assert rc == 0 and decode(buf, 0)["tiled"] == 0 and decode(buf, 1)["tiled"] == 1
    assert g.n_plain == 100 and g.ntiles > 0
    t = _lib.fof_tune()
    t.flags = _lib.FOF_TUNE_NO_TILES
    rc, g, _ = plan([100, 40000], [(3.0, 0.4), (40.0, 0.4)], tune=t)
    assert rc == 0 and g.n_plain == 40100 and g.ntiles == 0


def test_static_workspace_call_rejects_before_launch():
    """fof_find_groups_static checks its arguments and the plan's size against the static
    workspace on the host, before it touches a device."""
    L = lib()
    box = _lib.fof_box((ctypes.c_double * 3)(64.0, 64.0, 64.0), 0.4)
    bp = ctypes.byref(box)
    p = ctypes.c_void_p(0x100000)            # never dereferenced: every call below fails first
    args = lambda n, **kw: [kw.get("box", bp), n, None, kw.get("pos", p), 20, kw.get("vel"),
                            kw.get("cap", 10), kw.get("root", p), kw.get("gid", p),
                            kw.get("ng", p), kw.get("sizes", p), kw.get("com", p),
                            kw.get("vmean"), kw.get("sigv"), kw.get("status", p), None]
    f = L.fof_find_groups_static
    assert f(*args(100, box=None)) == _lib.FOF_EINVAL
    assert f(*args(-1)) == _lib.FOF_EINVAL
    assert f(*args(100, pos=None)) == _lib.FOF_EINVAL
    assert f(*args(100, root=None)) == _lib.FOF_EINVAL
    assert f(*args(100, gid=None)) == _lib.FOF_EINVAL
    assert f(*args(100, ng=None)) == _lib.FOF_EINVAL
    assert f(*args(100, status=None)) == _lib.FOF_EINVAL
    assert f(*args(100, cap=-1)) == _lib.FOF_EINVAL
    assert f(*args(100, com=None)) == _lib.FOF_EINVAL
    assert f(*args(100, vmean=p)) == _lib.FOF_EINVAL                   # vmean without vel
    assert f(*args(100, vel=p, vmean=p)) == _lib.FOF_EINVAL            # sigv missing
    bad = _lib.fof_box((ctypes.c_double * 3)(64.0, 64.0, 64.0), 40.0)  # 2b > L
    assert f(*args(100, box=ctypes.byref(bad))) == _lib.FOF_EINVAL
    # a plan larger than the static workspace: refused on the host
    big = _lib.fof_box((ctypes.c_double * 3)(512.0, 512.0, 512.0), 0.2)
    assert f(*args(3_000_000, box=ctypes.byref(big))) == _lib.FOF_ENOMEM
    cnt = (ctypes.c_int64 * 1)(3_000_000)
    g = _lib.fof_grid()
    assert L.fof_workspace_bytes(1, cnt, ctypes.byref(big), None, ctypes.byref(g), None, 0) == 0
    assert g.ws_bytes > _lib.FOF_STATIC_SCRATCH_BYTES


def test_cell_factor_scales_the_coarse_side_of_every_box():
    """fof_tune.cell_factor: the coarse side is that many of each box's own mean spacings."""
    L = lib()
    counts = (ctypes.c_int64 * 2)(64 ** 3, 32 ** 3)
    boxes = (_lib.fof_box * 2)()
    for k, side in enumerate((64.0, 32.0)):            # mean spacing 1.0 in both
        boxes[k].L[:] = [side] * 3
        boxes[k].b = 0.45                              # clique cells allow sides up to 2.59
    g = _lib.fof_grid()
    for factor, per_axis in ((0.0, (64, 32)), (1.0, (64, 32)), (2.0, (32, 16)),
                             (4.0, (25, 13))):         # 4 is capped: 10 clique cells per side
        t = _lib.fof_tune()
        t.cell_factor = factor
        assert L.fof_workspace_bytes(2, counts, boxes, ctypes.byref(t), ctypes.byref(g), None,
                                     0) == 0
        assert g.ncell == per_axis[0] ** 3 + per_axis[1] ** 3, factor
    for bad in (-1.0, float("nan"), float("inf")):
        t = _lib.fof_tune()
        t.cell_factor = bad
        assert L.fof_workspace_bytes(2, counts, boxes, ctypes.byref(t), ctypes.byref(g), None,
                                     0) == _lib.FOF_EINVAL
