"""Autotuner for the tuning knobs of fof_tune (coarse cell side, dense-cell threshold).

No knob changes any result; they only move work between the kernels.  The tuner times the
whole pipeline (build + link + groups) for a few candidates on the caller's own input and
keeps the fastest, cached in a JSON file keyed by device architecture, particle-count
bucket and the ratio of mean spacing to linking length.
"""
from __future__ import annotations

import json
import math
import os

import torch

from .fof import Plan

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "fof_mi355x", "tune.json")


def _key(n, L, b, device):
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", props.name)
    L3 = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
    spacing = (L3[0] * L3[1] * L3[2] / max(n, 1)) ** (1.0 / 3.0)
    return f"{arch}|n2^{int(math.log2(max(n, 1)))}|s/b={round(spacing / b, 1)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def candidates(n, L, b):
    L3 = [float(v) for v in (L if hasattr(L, "__len__") else (L, L, L))]
    spacing = (L3[0] * L3[1] * L3[2] / max(n, 1)) ** (1.0 / 3.0)
    out = []
    for f in (1.0, 1.5, 2.0):
        for thr in (16, 32, 64):
            out.append(dict(cell_side=max(f * spacing, 1.01 * b), dense_threshold=thr))
    return out


def time_pipeline(pos, L, b, tune, min_size=20, reps=3):
    plan = Plan([pos.shape[0]], [(L, b)], device=pos.device, tune=tune)
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


def autotune(pos, L, b, min_size=20, cache=DEFAULT_CACHE, reps=3, force=False, log=None):
    """Best tune dict for this input shape (cached)."""
    key = _key(pos.shape[0], L, b, pos.device)
    table = _load(cache) if cache else {}
    if key in table and not force:
        return table[key]["tune"]
    best, best_ms = None, float("inf")
    for tune in candidates(pos.shape[0], L, b):
        ms = time_pipeline(pos, L, b, tune, min_size, reps)
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
