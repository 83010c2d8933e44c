"""Launch-shape autotuner.

The edge and state autotuners are native (``vk_autotune_edges`` / ``vk_autotune_states`` in
libvk): they time every candidate launch setting on the caller's batch with HIP events (median of
7 launches; the edge tuner times its four fastest again over three interleaved rounds), set the
fastest on the robot handle, and keep it in a JSON cache keyed by the
workload's class (device, robot size, environment size, batch size), so that a later process
with the same class reuses it without timing.  The knobs of the persistent edge launch are the
workgroup size (waves per workgroup share one LDS copy of the environment), the workgroups per
compute unit (how many waves pull from the work queue at once) and the tickets per wave (how
many edges one queue ticket hands out); the knob of validate_states is its one- or two-pass
schedule.

``tune_batch`` tunes a mixed-robot batch, whose launch shape is fixed when the batch is created:
it creates one batch per candidate shape and keeps the fastest.
"""
from __future__ import annotations

import ctypes as C
import os

from . import EdgeBatch, _check, _dev_f32, _stream, lib

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "vk_autotune.json")
BLOCKS = (64, 128, 256, 512, 1024)
PER_CU = (1, 2, 4, 8)


def _path(cache):
    if not cache:
        return None
    os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
    return cache.encode()


def tune_edges(robot, env, qa, qb, n_states=None, resolution: float = 1.0 / 32.0,
               cache: str | None = DEFAULT_CACHE, force: bool = False):
    """Pick and set the robot's fastest edge launch for this batch (the launch shape, then the
    parts per edge); returns (block, per_cu, tickets)."""
    qa, qb = _dev_f32(qa, "qa"), _dev_f32(qb, "qb")
    ns = n_states.contiguous().data_ptr() if n_states is not None else None
    _check(lib().vk_autotune_edges(robot.handle, env.handle, qa.data_ptr(), qb.data_ptr(), ns,
                                   qa.shape[0], float(resolution), _path(cache), int(force),
                                   _stream()))
    return robot.get_edge_launch()


def tune_states(robot, env, q, cache: str | None = DEFAULT_CACHE, force: bool = False):
    """Pick and set the robot's fastest validate_states schedule for the SoA batch q [dof, N];
    returns (num, den)."""
    q = _dev_f32(q, "q")
    n = q.shape[1]
    _check(lib().vk_autotune_states(robot.handle, env.handle, q.data_ptr(), n, n, _path(cache),
                                    int(force), _stream()))
    return robot.get_states_split()


def tune_batch(robots, envs, sets, qa, qb, out, resolution: float = 1.0 / 32.0, reps: int = 7):
    """Create the mixed-robot batch with every candidate launch shape, time its replays (median
    of ``reps`` after one untimed replay) and return (fastest batch, {block, per_cu, ms})."""
    import torch
    best = None
    for block in BLOCKS:
        for per_cu in PER_CU:
            if block * per_cu > 2048:
                continue
            b = EdgeBatch(robots, envs, sets, resolution=resolution, block=block, per_cu=per_cu)
            b.run(qa, qb, out)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            ev[0].record()
            for r in range(reps):
                b.run(qa, qb, out)
                ev[r + 1].record()
            torch.cuda.synchronize()
            ms = sorted(ev[r].elapsed_time(ev[r + 1]) for r in range(reps))[reps // 2]
            if best is None or ms < best[0]:
                best = (ms, block, per_cu, b)
    ms, block, per_cu, b = best
    return b, {"block": block, "per_cu": per_cu, "ms": ms}


__all__ = ["tune_edges", "tune_states", "tune_batch", "DEFAULT_CACHE"]
