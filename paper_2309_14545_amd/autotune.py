"""Launch-shape autotuner for the persistent edge launch.

The persistent kernel's schedule has two knobs (``vk_set_edge_launch``): the workgroup size
(waves per workgroup share one LDS copy of the environment) and the number of workgroups per
compute unit (how many waves pull from the work queue at once).  ``tune_edges`` times every
candidate on the caller's batch with HIP events, keeps the fastest, and records it in a JSON
cache keyed by device and workload class (robot size, environment size, batch size), so a later
process with the same class reuses it without timing.
"""
from __future__ import annotations

import json
import os
import time

from . import get_edge_launch, set_edge_launch, validate_edges, set_states_split, validate_states

BLOCKS = (64, 128, 256, 512, 1024)
PER_CU = (1, 2, 4, 8)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "vk_autotune.json")


def _bucket(x: int) -> int:
    """Power-of-two bucket of a size (workload classes, not exact sizes)."""
    b = 1
    while b < x:
        b *= 2
    return b


def workload_key(robot, env, n_edges: int) -> str:
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device()).replace(" ", "_")
    prims = sum(env.counts.values())
    return f"{dev}|dof{robot.dof}|s{_bucket(robot.n_spheres)}|p{_bucket(max(prims, 1))}|e{_bucket(n_edges)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(robot, env, qa, qb, out, resolution, reps):
    import torch
    validate_edges(robot, env, qa, qb, resolution=resolution, out=out)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        validate_edges(robot, env, qa, qb, resolution=resolution, out=out)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def tune_edges(robot, env, qa, qb, resolution: float = 1.0 / 32.0, reps: int = 3,
               cache: str | None = DEFAULT_CACHE, force: bool = False, log=None):
    """Pick and apply the fastest (block, per-CU) for this batch; returns a result dict."""
    import torch
    key = workload_key(robot, env, qa.shape[0])
    data = _load(cache) if cache else {}
    if not force and key in data:
        block, per_cu = data[key]["block"], data[key]["per_cu"]
        set_edge_launch(block, per_cu)
        return {"key": key, "block": block, "per_cu": per_cu, "ms": data[key]["ms"], "cached": True}
    out = torch.empty(qa.shape[0], dtype=torch.uint8, device=qa.device)
    results = []
    t0 = time.perf_counter()
    for block in BLOCKS:
        for per_cu in PER_CU:
            if block * per_cu > 2048:          # more waves than a CU holds
                continue
            set_edge_launch(block, per_cu)
            ms = _time(robot, env, qa, qb, out, resolution, reps)
            results.append((ms, block, per_cu))
            if log:
                log(f"autotune {key}: block {block} per_cu {per_cu}: {ms:.3f} ms")
    ms, block, per_cu = min(results)
    set_edge_launch(block, per_cu)
    if cache:
        data = _load(cache)
        data[key] = {"block": block, "per_cu": per_cu, "ms": ms,
                     "candidates": [[b, p, round(m, 4)] for m, b, p in sorted(results)]}
        _save(cache, data)
    return {"key": key, "block": block, "per_cu": per_cu, "ms": ms, "cached": False,
            "tuning_s": time.perf_counter() - t0, "candidates": len(results)}


def tune_batch(make_batch, reps: int = 3, log=None):
    """Pick the fastest (block, per-CU) for a mixed-robot batch.  ``make_batch()`` builds an
    EdgeBatch under the current launch setting (its HIP graph captures that setting).
    Returns (batch, result)."""
    import torch
    best = None
    for block in BLOCKS:
        for per_cu in PER_CU:
            if block * per_cu > 2048:
                continue
            set_edge_launch(block, per_cu)
            b = make_batch()
            b.run()
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(reps):
                b.run()
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / reps
            if log:
                log(f"autotune batch: block {block} per_cu {per_cu}: {ms:.3f} ms")
            if best is None or ms < best[0]:
                best = (ms, block, per_cu, b)
    ms, block, per_cu, b = best
    set_edge_launch(block, per_cu)
    return b, {"block": block, "per_cu": per_cu, "ms": ms}


SPLITS = ((0, 1), (1, 3), (1, 2), (2, 3))


def tune_states(robot, env, q, reps: int = 3, log=None):
    """Pick and apply the fastest validate_states schedule (one pass, or two passes split after
    1/3, 1/2 or 2/3 of the link steps) for this batch; flags are the same for all of them."""
    import torch
    results = []
    for num, den in SPLITS:
        set_states_split(num, den)
        validate_states(robot, env, q)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            validate_states(robot, env, q)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        results.append((ms, num, den))
        if log:
            log(f"autotune states: split {num}/{den}: {ms:.3f} ms")
    ms, num, den = min(results)
    set_states_split(num, den)
    return {"split": [num, den], "ms": ms}


__all__ = ["tune_edges", "tune_batch", "tune_states", "workload_key", "get_edge_launch"]
