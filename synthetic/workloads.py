"""Workload table: seeded robots, scenes and batches of configurations / edges / trajectories.

Every random stream is derived from one root seed and a (workload, component) key, so a
component (e.g. the 7-DoF robot) is identical wherever it is reused.  Configurations are drawn
in FP64 and cast to FP32; the FP32 values are canonical for both the GPU path and the oracle.

Workloads (sizes are the defaults; tests pass smaller ``n``):

=================  ============================================================================
``states7``        7-DoF chain, 6 spheres/link (42), every pruned non-adjacent pair; 32 spheres
                   + 8 boxes in a 2 m cube; 4,096 uniform states (SoA [dof][N])
``edges7_shelf``   the same 7-DoF robot in the shelf scene (100 boxes + 50 capsules);
                   65,536 edges with endpoints uniform in the limits
``edges7_shelf_near`` the same robot and batch with the shelf units at U[0.55, 1.1] m (each panel
                   kept out of the base's keep-out ball on its own), within the arm's reach
``edges8_shelf``   8-DoF chain, 4 base + 8x7 spheres (60), 400 pairs; shelf scene; 65,536 edges
``edges8p_shelf``  prismatic lift (0-0.4 m) + 7-DoF arm, 4 torso + 7x6 spheres (46), 400 pairs;
                   shelf scene; 65,536 edges uniform in each joint's range
``states14_cloud`` two 7-DoF arms on a torso (120 spheres, 1,500 pairs); 300 spheres + a
                   20,000-point cloud; 2^20 uniform states
``cost7``          the states7 robot and scene; 4,096 trajectories x 64 waypoints
``prm7_shelf``     the 7-DoF robot in the shelf scene; 8,192 roadmap samples, k = 10
``shortcut7_shelf`` the 7-DoF robot in the shelf scene; 4,096 jittered straight paths of 32
                   waypoints, 8 random shortcut candidates per path (32,768 edges)
``mixed``          1,024 edge sets over the 7/8/14-DoF robots, lognormal(4, 1) edges per set,
                   a random scene of 50-300 primitives per set
=================  ============================================================================
"""
from __future__ import annotations

import zlib

import numpy as np

from .robots import chain_robot, bimanual_robot, lift_arm_robot, Q_LIMIT
from .scenes import cube_scene, shelf_scene, point_cloud_scene, random_scene

ROOT_SEED = 230914545
TORSO_MOUNTS = ((0.0, 0.25, 0.5), (0.0, -0.25, 0.5), (0.0, 0.0, 0.0))


def rng(workload: str, component: str) -> np.random.Generator:
    key = (zlib.crc32(workload.encode()), zlib.crc32(component.encode()))
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=key))


def uniform_states(g: np.random.Generator, dof: int, n: int, limit: float = Q_LIMIT,
                   layout: str = "soa") -> np.ndarray:
    """n configurations uniform in [-limit, limit]^dof; SoA [dof][n] by default."""
    q = g.uniform(-limit, limit, (n, dof)).astype(np.float32)
    return np.ascontiguousarray(q.T) if layout == "soa" else q


def uniform_edges(g: np.random.Generator, dof: int, n: int, limit: float = Q_LIMIT,
                  lo=None, hi=None):
    """n edges; endpoints uniform in the limits (per joint when lo/hi are given); AoS [n][dof]
    each."""
    lo = -limit if lo is None else np.asarray(lo, np.float64)
    hi = limit if hi is None else np.asarray(hi, np.float64)
    qa = g.uniform(lo, hi, (n, dof)).astype(np.float32)
    qb = g.uniform(lo, hi, (n, dof)).astype(np.float32)
    return qa, qb


def trajectories(g: np.random.Generator, dof: int, n_traj: int, n_way: int = 64,
                 limit: float = Q_LIMIT, sigma: float = 0.05) -> np.ndarray:
    """Straight-line trajectories with jittered interior waypoints; SoA [dof][n_traj*n_way]."""
    a = g.uniform(-limit, limit, (n_traj, 1, dof))
    b = g.uniform(-limit, limit, (n_traj, 1, dof))
    s = np.linspace(0.0, 1.0, n_way)[None, :, None]
    q = a + s * (b - a)
    q[:, 1:-1, :] += g.normal(0.0, sigma, (n_traj, n_way - 2, dof))
    q = np.clip(q, -limit, limit).reshape(n_traj * n_way, dof).astype(np.float32)
    return np.ascontiguousarray(q.T)


def shortcut_pairs(g: np.random.Generator, n_paths: int, n_way: int, per_path: int) -> np.ndarray:
    """Random shortcut candidates (i < j, j - i >= 2) between waypoints of each path, as node
    index pairs; waypoint w of path p is node p * n_way + w."""
    i = g.integers(0, n_way - 2, (n_paths, per_path))
    j = i + 2 + np.floor(g.random((n_paths, per_path)) * (n_way - 2 - i)).astype(np.int64)
    base = (np.arange(n_paths) * n_way)[:, None]
    return np.stack([base + i, base + j], axis=-1).reshape(-1, 2).astype(np.int32)


def robot7():
    return chain_robot(rng("robot7", "robot"), dof=7, spheres_per_link=6)


def robot8p():
    return lift_arm_robot(rng("robot8p", "robot"), arm_dof=7, spheres_per_link=6, torso_spheres=4,
                          n_pairs=400)


def robot8():
    return chain_robot(rng("robot8", "robot"), dof=8, spheres_per_link=7, base_spheres=4,
                       n_pairs=400)


def robot14():
    return bimanual_robot(rng("robot14", "robot"), arm_dof=7, spheres_per_link=8,
                          torso_spheres=8, n_pairs=1500)


def _lognormal_counts(g, n_sets, mu=4.0, sigma=1.0):
    return np.maximum(1, np.floor(np.exp(g.normal(mu, sigma, n_sets)))).astype(np.int64)


def pack_edge_sets(w: dict, max_edges: int | None = None):
    """Concatenate a mixed workload's edge sets into flat FP32 qa / qb arrays.

    Returns (qa, qb, sets, total) with sets as (robot, env, float offset, n_edges, out offset)
    tuples in the layout of the mixed-batch C interface."""
    qa_parts, qb_parts, sets, off, out_off = [], [], [], 0, 0
    for k, (ri, ei, _) in enumerate(w["sets"]):
        a, b = w["qa"][k], w["qb"][k]
        if max_edges:
            a, b = a[:max_edges], b[:max_edges]
        qa_parts.append(a.reshape(-1))
        qb_parts.append(b.reshape(-1))
        sets.append((ri, ei, off, len(a), out_off))
        off += a.size
        out_off += len(a)
    qa = np.concatenate(qa_parts).astype(np.float32) if qa_parts else np.zeros(1, np.float32)
    qb = np.concatenate(qb_parts).astype(np.float32) if qb_parts else np.zeros(1, np.float32)
    return qa, qb, sets, out_off


def workload(name: str, n: int | None = None, variant: int = 0) -> dict:
    """Return a dict with the robot(s), scene(s) and batch of the named workload.

    ``n`` overrides the batch size (states, edges, trajectories or edge sets); ``variant``
    selects another seeded draw of the batch (used for repeated mixed batches).
    """
    if name == "states7":
        robot = robot7()
        env = cube_scene(rng("states7", "env"))
        q = uniform_states(rng("states7", "q"), robot["dof"], n or 4096)
        return {"name": name, "robot": robot, "env": env, "q": q}
    if name == "edges7_shelf":
        robot = robot7()
        env = shelf_scene(rng("shelf", "env"))
        qa, qb = uniform_edges(rng("edges7_shelf", "edges"), robot["dof"], n or 65536)
        return {"name": name, "robot": robot, "env": env, "qa": qa, "qb": qb}
    if name == "edges7_shelf_near":
        robot = robot7()
        env = shelf_scene(rng("shelf_near", "env"), radius=(0.55, 1.1), keepout="box")
        qa, qb = uniform_edges(rng("edges7_shelf", "edges"), robot["dof"], n or 65536)
        return {"name": name, "robot": robot, "env": env, "qa": qa, "qb": qb}
    if name == "edges8_shelf":
        robot = robot8()
        env = shelf_scene(rng("shelf", "env"))
        qa, qb = uniform_edges(rng("edges8_shelf", "edges"), robot["dof"], n or 65536)
        return {"name": name, "robot": robot, "env": env, "qa": qa, "qb": qb}
    if name == "edges8p_shelf":
        # prismatic lift + 7-DoF arm in the shelf scene; endpoints uniform in each joint's range
        robot = robot8p()
        env = shelf_scene(rng("shelf", "env"))
        qa, qb = uniform_edges(rng("edges8p_shelf", "edges"), robot["dof"], n or 65536,
                               lo=robot["q_lo"], hi=robot["q_hi"])
        return {"name": name, "robot": robot, "env": env, "qa": qa, "qb": qb}
    if name == "states14_cloud":
        robot = robot14()
        env = point_cloud_scene(rng("states14_cloud", "env"), mounts=TORSO_MOUNTS)
        q = uniform_states(rng("states14_cloud", "q"), robot["dof"], n or (1 << 20))
        return {"name": name, "robot": robot, "env": env, "q": q}
    if name == "prm7_shelf":
        # PRM roadmap: samples uniform in the limits, each joined to its k nearest
        robot = robot7()
        env = shelf_scene(rng("shelf", "env"))
        nodes = uniform_states(rng("prm7_shelf", "nodes"), robot["dof"], n or 8192, layout="aos")
        return {"name": name, "robot": robot, "env": env, "nodes": nodes, "k": 10}
    if name == "shortcut7_shelf":
        # shortcut candidates on many jittered straight-line paths of 32 waypoints each
        robot = robot7()
        env = shelf_scene(rng("shelf", "env"))
        n_paths, n_way = n or 4096, 32
        way = trajectories(rng("shortcut7_shelf", "paths"), robot["dof"], n_paths, n_way)
        nodes = np.ascontiguousarray(way.T)
        pairs = shortcut_pairs(rng("shortcut7_shelf", "pairs"), n_paths, n_way, 8)
        return {"name": name, "robot": robot, "env": env, "nodes": nodes, "pairs": pairs}
    if name == "cost7":
        robot = robot7()
        env = cube_scene(rng("states7", "env"))
        n_traj = n or 4096
        q = trajectories(rng("cost7", "traj"), robot["dof"], n_traj)
        return {"name": name, "robot": robot, "env": env, "q": q, "n_traj": n_traj}
    if name == "mixed":
        robots = [robot7(), robot8(), robot14()]
        n_sets = n or 1024
        tag = "mixed" if variant == 0 else f"mixed{variant}"
        g = rng(tag, "sets")
        which = g.integers(0, 3, n_sets)
        counts = _lognormal_counts(g, n_sets)
        envs, sets, qa, qb = [], [], [], []
        for k in range(n_sets):
            r = robots[which[k]]
            mounts = TORSO_MOUNTS if r["dof"] == 14 else ((0.0, 0.0, 0.0),)
            envs.append(random_scene(rng(tag, f"env{k}"), mounts=mounts))
            a, b = uniform_edges(rng(tag, f"edges{k}"), r["dof"], int(counts[k]))
            qa.append(a)
            qb.append(b)
            sets.append((int(which[k]), k, int(counts[k])))
        return {"name": name, "robots": robots, "envs": envs, "sets": sets, "qa": qa, "qb": qb}
    raise KeyError(name)
