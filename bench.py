"""Benchmark of the Friends-of-Friends hot path on one MI355X.

A step is one pass of the whole hot path over the resident input: fof_build_grid (cell
binning) + fof_link (labels) + fof_groups (catalogue with centres of mass).  The default
workload is the 512^3 Zel'dovich box with 50,000 NFW clumps (L = 512, b = 0.2, min size 20).

Prints ONE JSON line (rank 0) with the metric, the per-stage times, the HBM roofline of the
link pass and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--config 2] [--no-cpu-baseline]

--config 5 runs the same recipe at 1024^3 (1.07e9 particles, L = 1024, 400,000 clumps) in
one box on one GPU; drawing it takes minutes and about 80 GB of host memory.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per particle (what the method must move): link reads the sorted
# position (12) and the original index (4) and writes one label (4).
LINK_BYTES_PER_PARTICLE = 20
BUILD_BYTES_PER_PARTICLE = 28
GROUPS_BYTES_PER_PARTICLE = 20


# The link stage (fof_link) as launched on the benchmark workload: its kernels, in order.
LINK_STAGE = "fof_link: k_fill, k_dense_small/big<0> (components), k_dense_small/big<1> " \
             "(dense pairs), k_link_tiled, k_link_edges, k_link_windows, k_link, " \
             "k_dense_small/big<2> (sparse-dense), k_compress"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "link_stage_traffic_zeldovich-nfw-512.txt")


def kernel_digest():
    """SHA-256 over the HIP sources and the ABI header: recorded HBM traffic is reported only
    while the kernels it was measured on are unchanged."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2510_26851_amd", "csrc", "*"))) + \
        [os.path.join(ROOT, "include", "fof.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload, tune):
    """HBM bytes per link-stage launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE record, or
    None when there is none for this workload and these kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.strip().split("=", 1) for l in f if "=" in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("workload") != workload or kv.get("kernel_digest") != kernel_digest() or \
            kv.get("tune") != json.dumps(tune, sort_keys=True):
        return None
    return float(kv["hbm_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(box, zmax):
    """The oracle as it stands on the particles with z < zmax, treated as a periodic
    L x L x zmax box (same density, clumps and linking length): labels + groups, first with
    the multi-threaded labelling (OpenMP, the runtime's default thread count), then
    single-threaded."""
    import numpy as np

    import oracle

    sel = box.pos[:, 2] < np.float32(zmax)
    pos = np.ascontiguousarray(box.pos[sel])
    L = (box.L[0], box.L[1], float(zmax))
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    root, _ = oracle.fof_par(pos, L, box.b)
    oracle.groups(pos, root, L, box.min_size)
    dt_par = time.perf_counter() - t0
    t0 = time.perf_counter()
    root1, _ = oracle.fof(pos, L, box.b)
    oracle.groups(pos, root1, L, box.min_size)
    dt1 = time.perf_counter() - t0
    if not np.array_equal(root, root1):
        raise SystemExit("the two oracle forms disagree")
    return dict(value=pos.shape[0] / dt_par / 1e6, unit="Mparticles/s", cores=threads,
                kind="oracle", seconds=round(dt_par, 3), cpu=cpu_model(),
                affinity_cpus=len(os.sched_getaffinity(0)),
                single_thread={"value": pos.shape[0] / dt1 / 1e6, "cores": 1,
                               "seconds": round(dt1, 3)},
                sample=f"particles with z < {zmax} of the same box ({pos.shape[0]}), "
                       f"treated as a periodic {L[0]:g}x{L[1]:g}x{L[2]:g} box; labels "
                       f"(pair enumeration on {threads} OpenMP threads, shared union-find) "
                       f"+ groups (serial)")


def copy_bandwidth(torch, dev, nbytes=2 << 30):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 5 / 1e3
    del a, b
    return 2 * nbytes / t / 1e9


METRIC = "Mparticles/s end-to-end FoF at 512\u00b3 + % HBM peak; batched REINFORCE samples/s"


def reinforce_rate(torch, dev, reps):
    """Stochastic linking of the 128^3 velocity box, timed per batch of K = 64 samples: the
    candidate edges, the K sampled graphs and their components (fof_link with the sample),
    every sample's halos (fof_groups with the sample: sizes and centres), the loss of each
    sample (sum of squared halo sizes, from the tables) and the score-function gradient
    (fof_backward FOF_SCORE).  Beside it the same 64 graphs drawn by 64 sequential calls of
    one sample each (s_first = 0..63: edges rebuilt every call), their halos and losses, then
    one gradient over the 64 losses; both give the same losses exactly."""
    import workloads as W
    from paper_2510_26851_amd.reinforce import Sampler, sum_sq_sizes

    box = W.config3()
    K = W.CONFIG3_K
    tau = W.CONFIG3_TAU_FRAC * box.b
    pos = torch.from_numpy(box.pos).to(dev)
    smp = Sampler(pos, box.L, box.b, tau, K, W.REINFORCE_SEED)
    smp.sample()                     # fits the edge capacity (one read-back)
    # group tables sized from this first draw (the most groups of any sample, plus a
    # quarter): a caller's choice that keeps the tables and the loss over them small; an
    # overflow in the timed draws would set the status bit checked below
    first = smp.groups(2)
    cap = int(first["n_groups"].max().item()) * 5 // 4 + 1024
    halos = smp.groups(2, cap=cap)
    gp = torch.empty((box.n, 3), dtype=torch.float32, device=dev)

    def batched():
        smp.sample()
        h = smp.groups(2, cap=halos["cap"], out=halos)
        smp.grad(sum_sq_sizes(h), out=gp)

    one = Sampler(pos, box.L, box.b, tau, 1, W.REINFORCE_SEED, edge_cap=smp.S.edge_cap)
    seq_losses = torch.empty(K, dtype=torch.float64, device=dev)
    out1 = {}

    def sequential():
        for k in range(K):
            one.S.s_first = k
            one.sample()
            h = one.groups(2, cap=halos["cap"], out=out1)
            out1.update(h)
            seq_losses[k:k + 1] = sum_sq_sizes(h)
        smp.grad(seq_losses, out=gp)

    stream = torch.cuda.current_stream()
    res = {}
    for name, fn, r in (("batched", batched, reps), ("sequential", sequential, max(2, reps // 4))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(r):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / r
        res[name] = {"ms_per_batch": round(ms, 4), "samples_per_s": round(K / (ms / 1e3), 1),
                     "reps": r}
    if smp.plan.status() != 0 or one.plan.status() != 0:
        raise SystemExit("device status set in the REINFORCE leg")
    smp.sample()
    same = bool(torch.equal(sum_sq_sizes(smp.groups(2, out=halos)), seq_losses))
    if not same:
        raise SystemExit("batched and sequential REINFORCE losses differ")
    return {"workload": box.name, "n": box.n, "K": K, "tau": tau,
            "edges": int(smp.n_edges.item()), "ms_per_batch": res["batched"]["ms_per_batch"],
            "samples_per_s": res["batched"]["samples_per_s"],
            "sequential": res["sequential"], "same_losses": same,
            "table_cap": halos["cap"],
            "timed": "batched: fof_link(sample K=64) + fof_groups(sample) + loss from the halo "
                     "tables + fof_backward(FOF_SCORE); sequential: 64 x [fof_link(sample K=1, "
                     "s_first=k) + fof_groups(sample) + loss] + one fof_backward(FOF_SCORE)"}


def batched_rate(torch, dev, reps, tune=None):
    """The batched workload: 256 periodic boxes of log-uniform sizes (16^3 to 128^3 particles,
    clumped, b = 0.2 mean spacing per box, min size 20).  Three forms of the same pipeline
    (fof_build_grid + fof_link + fof_groups), timed with HIP events on the launch stream:
      graph:   the whole batch as one plan, captured once in a hipGraph and replayed;
      batched: the same plan launched eagerly;
      looped:  one plan per box, the boxes one after another (the single-box path).
    The looped labels and group counts must equal the batched ones exactly.  Unless given,
    the tuning (cell size per box spacing, dense threshold, block) is the autotuner's choice
    for this batch."""
    import numpy as np

    import workloads as W
    from paper_2510_26851_amd import Plan

    from paper_2510_26851_amd.tune import autotune_batch

    boxes = W.config4()
    counts = [bx.n for bx in boxes]
    n = int(sum(counts))
    pos = torch.from_numpy(np.concatenate([bx.pos for bx in boxes])).to(dev)
    if tune is None:  # tuned on this input (no cache), the same choice for every form
        t0 = time.perf_counter()
        tune = autotune_batch(pos, counts, [(bx.L, bx.b) for bx in boxes], 20, cache=None,
                              reps=2)
        log(f"batch tuned in {time.perf_counter() - t0:.1f}s: {tune}")
    plan = Plan(counts, [(bx.L, bx.b) for bx in boxes], device=dev, tune=tune)
    root = torch.empty(n, dtype=torch.int32, device=dev)
    out = dict(group_id=torch.empty(n, dtype=torch.int32, device=dev),
               n_groups=torch.empty(1, dtype=torch.int32, device=dev),
               sizes=torch.empty(n, dtype=torch.int32, device=dev),
               com=torch.empty((n, 3), dtype=torch.float64, device=dev))

    def step():
        plan.build_grid(pos)
        plan.link(root)
        plan.groups(20, out=out)

    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    views = [pos[offs[k]:offs[k + 1]] for k in range(len(boxes))]
    plans = [Plan([bx.n], [(bx.L, bx.b)], device=dev, tune=tune) for bx in boxes]
    roots = [torch.empty(bx.n, dtype=torch.int32, device=dev) for bx in boxes]
    outs = [dict(group_id=torch.empty(bx.n, dtype=torch.int32, device=dev),
                 n_groups=torch.empty(1, dtype=torch.int32, device=dev),
                 sizes=torch.empty(bx.n, dtype=torch.int32, device=dev),
                 com=torch.empty((bx.n, 3), dtype=torch.float64, device=dev)) for bx in boxes]

    def looped():
        for p, v, r, o in zip(plans, views, roots, outs):
            p.build_grid(v)
            p.link(r)
            p.groups(20, out=o)

    stream = torch.cuda.current_stream()
    step()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        step()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()

    res = {}
    for name, fn, r in (("graph", graph.replay, reps), ("batched", step, reps),
                        ("looped", looped, max(2, reps // 2))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(r):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / r
        res[name] = {"ms": round(ms, 4), "mparticles_per_s": round(n / (ms / 1e3) / 1e6, 1),
                     "reps": r}
    if plan.status() != 0 or any(p.status() != 0 for p in plans):
        raise SystemExit("device status set in the batched leg")
    graph.replay()
    looped()
    torch.cuda.synchronize()
    same = all(torch.equal(root[offs[k]:offs[k + 1]] - int(offs[k]), roots[k])
               for k in range(len(boxes)))
    ng_loop = sum(int(o["n_groups"].item()) for o in outs)
    same = same and ng_loop == int(out["n_groups"].item())
    if not same:
        raise SystemExit("batched and looped labels differ")
    return {"workload": f"{len(boxes)} clumped boxes, 16^3-128^3 particles each",
            "n": n, "boxes": len(boxes), "groups": ng_loop, "tune": tune,
            "graph": res["graph"], "batched": res["batched"], "looped": res["looped"],
            "same_labels": same,
            "timed": "fof_build_grid + fof_link + fof_groups over all boxes: one plan replayed "
                     "as a hipGraph, the same plan eagerly, and one plan per box in a loop"}


def stream_rate(torch, pos, box, in_core_root, in_core_ws, reps=3, nslab=16):
    """Streaming labels of the same box in z-slabs (fof_link_stream): per-call time (HIP
    events on the launch stream), its workspace against the in-core plan's, and the labels
    checked against the in-core labels of the timed step."""
    from paper_2510_26851_amd import Stream

    st = Stream(pos, box.L, box.b, nslab=nslab)
    root = torch.empty_like(in_core_root)
    st.labels(root)
    torch.cuda.synchronize()
    if st.status() != 0 or not torch.equal(root, in_core_root):
        raise SystemExit("streaming labels differ from the in-core labels")
    stream = torch.cuda.current_stream()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        st.labels(root)
    e.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    return dict(workload=box.name, slabs=nslab, ms=round(ms, 3),
                mparticles_per_s=round(box.n / (ms / 1e3) / 1e6, 1),
                workspace_GB=round(st.ws_bytes / 1e9, 3),
                in_core_workspace_GB=round(in_core_ws / 1e9, 3),
                workspace_fraction=round(st.ws_bytes / in_core_ws, 4), same_labels=True,
                timed="fof_link_stream: per slab, gather + fof_build_grid + fof_link + fusion")


def decorated_rate(torch, plan, pos, out, cap, ng, stream, workload, reps=10):
    """Decorated frozen assignment on the groups of the last step: per-call time of the
    position dispersion (fof_group_dispersion) and of its gradient (fof_backward_dispersion,
    which adds into grad_pos), HIP events on the launch stream."""
    res = dict(out, cap=cap)
    sig = torch.empty(cap, dtype=torch.float64, device=pos.device)
    grad = torch.zeros_like(pos)
    gen = torch.Generator(device=pos.device).manual_seed(1)
    g_sigx = torch.randn(max(ng, 1), dtype=torch.float64, device=pos.device, generator=gen)
    G = min(ng, cap)

    def fwd():
        plan.dispersion(res, sigx=sig)

    def bwd():
        plan.backward_dispersion(pos, out["group_id"], G, out["sizes"], out["com"], sig, g_sigx,
                                 grad)

    times = {}
    for name, fn in (("dispersion_ms", fwd), ("backward_ms", bwd)):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        times[name] = round(a.elapsed_time(b) / reps, 4)
    return dict(workload=workload, groups=G, **times,
                timed="fof_group_dispersion; fof_backward_dispersion (adds into grad_pos)")


def subhalo_rate(torch, dev, reps=5):
    """Six-dimensional sub-halo pass over the hosts of a phase-space box: 2000 hosts of three
    sub-clumps (30-400 members each) in a 96^3 box with 2M background particles, b = 0.2,
    min size 20, factors 0.04 and 1.0, b6 = 1.  Times fof_subhalo alone (HIP events on the
    launch stream) and counts the member pairs it tests."""
    import numpy as np

    import workloads as W
    from paper_2510_26851_amd import Plan, trim

    L, b = 96.0, 0.2
    pos, vel = W.phase_space_hosts(2000, L, W.SEED_BASE + 200, n_background=2_000_000)
    tp, tv = torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev)
    plan = Plan([pos.shape[0]], [(L, b)], device=dev)
    plan.build_grid(tp)
    plan.link()
    res = trim(plan.groups(20))
    G = int(res["n_groups"])
    nx = torch.full((G,), 0.04, dtype=torch.float64, device=dev)
    nv = torch.ones(G, dtype=torch.float64, device=dev)
    sub = torch.empty(pos.shape[0], dtype=torch.int32, device=dev)
    plan.subhalo(tp, tv, res["group_id"], G, res["sizes"], nx, nv, 1.0, sub=sub)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        plan.subhalo(tp, tv, res["group_id"], G, res["sizes"], nx, nv, 1.0, sub=sub)
    e.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(e) / reps
    m = res["sizes"].cpu().numpy().astype(np.float64)
    pairs = float(np.sum(m * (m - 1) / 2))
    s = sub.cpu().numpy()
    return dict(workload=f"phase-space hosts: 2000 x 3 sub-clumps + 2M background, L={L:g}",
                n=int(pos.shape[0]), hosts=G, subhalos=int(np.unique(s[s >= 0]).size),
                ms=round(ms, 4), pairs=int(pairs), gpairs_per_s=round(pairs / ms / 1e6, 2),
                timed="fof_subhalo (scatter into hosts, all-pairs 6-D test, labels)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-zmax", type=float, default=0.0,
                    help="CPU sample: particles with z < zmax (0 = about 16.8M particles)")
    ap.add_argument("--cell-side", type=float, default=0.0, help="coarse cell side (0 = default)")
    ap.add_argument("--dense-threshold", type=int, default=0, help="0 = default, <0 = off")
    ap.add_argument("--block", type=int, default=0, help="threads per block (0 = default)")
    ap.add_argument("--no-tiles", action="store_true", help="link without LDS tiles")
    ap.add_argument("--no-reinforce", action="store_true")
    ap.add_argument("--reinforce-reps", type=int, default=20)
    ap.add_argument("--no-subhalo", action="store_true")
    ap.add_argument("--no-decorated", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--cache-dir", default="",
                    help="store / reuse the drawn positions here (.npy; none by default)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2510_26851_amd import Plan

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    box = W.make(args.config, progress=log, cache_dir=args.cache_dir or None)
    log(f"generated {box.name}: n={box.n} L={box.L} b={box.b} in {time.perf_counter() - t0:.1f}s")

    pos = torch.from_numpy(box.pos).to(dev)
    vel = torch.from_numpy(box.vel).to(dev) if box.vel is not None else None
    tune = dict(cell_side=args.cell_side, dense_threshold=args.dense_threshold, block=args.block,
                flags=1 if args.no_tiles else 0)
    plan = Plan([box.n], [(box.L, box.b)], device=dev, tune=tune)
    root = torch.empty(box.n, dtype=torch.int32, device=dev)
    cap = box.n
    out = dict(group_id=torch.empty(box.n, dtype=torch.int32, device=dev),
               n_groups=torch.empty(1, dtype=torch.int32, device=dev),
               sizes=torch.empty(cap, dtype=torch.int32, device=dev),
               com=torch.empty((cap, 3), dtype=torch.float64, device=dev))
    if vel is not None:
        out["vmean"] = torch.empty((cap, 3), dtype=torch.float64, device=dev)
        out["sigv"] = torch.empty(cap, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]

    def step(e=None):
        if e:
            e[0].record(stream)
        plan.build_grid(pos)
        if e:
            e[1].record(stream)
        plan.link(root)
        if e:
            e[2].record(stream)
        plan.groups(box.min_size, vel=vel, cap=cap, out=out)
        if e:
            e[3].record(stream)

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {k + 1}/{args.warmup} done")
    if plan.status() != 0:
        raise SystemExit(f"device status {plan.status()}")
    ng = int(out["n_groups"].item())

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {wall:.3f}s")

    st = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                   for e in ev])
    build_ms, link_ms, groups_ms = (float(np.median(st[:, j])) for j in range(3))
    link_mean_ms = float(np.mean(st[:, 1]))
    ms_per_step = wall / args.steps * 1e3
    value = box.n / (ms_per_step / 1e3) / 1e6
    achieved = LINK_BYTES_PER_PARTICLE * box.n / (link_mean_ms / 1e3) / 1e9
    copy_gbs = copy_bandwidth(torch, dev)
    log(f"copy bandwidth {copy_gbs:.0f} GB/s")
    traffic = recorded_traffic(box.name, tune)

    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mparticles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": box.name, "n": box.n, "L": box.L[0], "b": box.b,
                   "min_size": box.min_size, "n_groups": ng, "tune": tune},
        "stages_ms": {"build_grid": round(build_ms, 4), "link": round(link_ms, 4),
                      "groups": round(groups_ms, 4)},
        "hbm_frac_end_to_end": round((BUILD_BYTES_PER_PARTICLE + LINK_BYTES_PER_PARTICLE +
                                      GROUPS_BYTES_PER_PARTICLE) * box.n /
                                     (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": {"kernel": LINK_STAGE, "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 4),
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "scaled by a 2 GiB copy)",
                     "algorithmic_GB_per_launch": round(LINK_BYTES_PER_PARTICLE * box.n / 1e9, 4),
                     "bytes_per_particle": LINK_BYTES_PER_PARTICLE,
                     "avg_ms": round(link_mean_ms, 4)},
        "hbm_peak_frac_link": round(achieved / HBM_PEAK_GBS, 4),
        "copy_gbs": round(copy_gbs, 1),
    }
    if not args.no_decorated:
        line["decorated"] = decorated_rate(torch, plan, pos, out, cap, ng, stream, box.name)
    if not args.no_stream:
        log("timing the streaming labels ...")
        line["stream"] = stream_rate(torch, pos, box, root, plan.ws_bytes)
    if not args.no_reinforce:
        log("timing batched REINFORCE ...")
        line["reinforce"] = reinforce_rate(torch, dev, args.reinforce_reps)
    if not args.no_batched:
        log("timing the batch of 256 boxes ...")
        line["batched"] = batched_rate(torch, dev, 10)
    if not args.no_subhalo:
        log("timing the sub-halo pass ...")
        line["subhalo"] = subhalo_rate(torch, dev)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        zmax = args.cpu_zmax or 64.0 * (512.0 / box.L[0]) * (512.0 / box.L[1])
        line["cpu_baseline"] = cpu_baseline(box, zmax)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
