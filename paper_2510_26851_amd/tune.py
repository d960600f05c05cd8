"""Autotuner for the knobs of fof_tune: coarse cell size (relative to each box's own mean
particle spacing, so one value suits a batch of boxes of different densities), the
dense-cell threshold, and the block shape of the per-particle kernels.

No knob changes any result; they only move work between the kernels.  The tuner times the
whole pipeline (build + link + groups) on the caller's own input, first over (cell factor,
dense threshold) at the default block, then over the block at the best pair, and keeps the
fastest.  Choices are cached in a JSON file keyed by device architecture, particle-count
bucket, number of boxes and the ratio of mean spacing to linking length.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from .fof import Plan

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "fof_mi355x", "tune.json")

CELL_FACTORS = (1.0, 1.25, 1.5, 2.0)
DENSE_THRESHOLDS = (16, 32, 64)
BLOCKS = (128, 256, 512)


def _L3(L):
    return [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]


def _key(counts, boxes, device):
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", props.name)
    n = int(sum(counts))
    ratios = []
    for c, (L, b) in zip(counts, boxes):
        L3 = _L3(L)
        if c > 0:
            ratios.append((L3[0] * L3[1] * L3[2] / c) ** (1.0 / 3.0) / b)
    ratio = float(np.median(ratios)) if ratios else 0.0
    nb = len(counts)
    nbk = 1 if nb == 1 else 2 ** int(math.ceil(math.log2(nb)))
    return f"{arch}|n2^{int(math.log2(max(n, 1)))}|boxes<={nbk}|s/b={round(ratio, 1)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def candidates():
    """Stage one: (cell factor, dense threshold) at the default block."""
    return [dict(cell_factor=f, dense_threshold=t) for f in CELL_FACTORS
            for t in DENSE_THRESHOLDS]


def time_pipeline(pos, counts, boxes, tune, min_size=20, reps=3):
    """Milliseconds per build + link + groups of the batch under `tune` (HIP events)."""
    plan = Plan(counts, boxes, device=pos.device, tune=tune)
    root = torch.empty(pos.shape[0], dtype=torch.int32, device=pos.device)

    def step():
        plan.build_grid(pos)
        plan.link(root)
        plan.groups(min_size, cap=1)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune_batch(pos, counts, boxes, min_size=20, cache=DEFAULT_CACHE, reps=3, force=False,
                   log=None):
    """Best tune dict for a batch of boxes (counts[k] particles in box k, boxes[k] = (L, b),
    pos the concatenated float32 [n, 3] positions on the GPU); cached."""
    counts = [int(c) for c in counts]
    key = _key(counts, boxes, pos.device)
    table = _load(cache) if cache else {}
    if key in table and not force:
        return table[key]["tune"]
    best, best_ms = None, float("inf")
    for tune in candidates():
        ms = time_pipeline(pos, counts, boxes, tune, min_size, reps)
        if log:
            log(f"tune {tune}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = tune, ms
    for blk in BLOCKS:
        tune = dict(best, block=blk)
        if blk == 256:  # the default block, already timed in stage one
            continue
        ms = time_pipeline(pos, counts, boxes, tune, min_size, reps)
        if log:
            log(f"tune {tune}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = tune, ms
    if cache:
        table[key] = dict(tune=best, ms=best_ms)
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


def autotune(pos, L, b, min_size=20, cache=DEFAULT_CACHE, reps=3, force=False, log=None):
    """Best tune dict for one box of side(s) L and linking length b (cached)."""
    return autotune_batch(pos, [pos.shape[0]], [(L, b)], min_size=min_size, cache=cache,
                          reps=reps, force=force, log=log)
