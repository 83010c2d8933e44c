"""Seeded synthetic environments made of primitives.

The method models obstacles as spheres, cylinders and cuboids (Sec. III-C).  The evaluation
scenes (tabletop, bookshelf, box and cage problems, Sec. IV) are not available here, so these
generators stand in for them:

* ``cube_scene``        random spheres and oriented boxes in a 2 m cube;
* ``shelf_scene``       shelf units (side panels, back panel, boards) in a half ring in front of
                        the base, with upright capsules and a few small boxes on the boards;
* ``point_cloud_scene`` random spheres plus a noisy sampled table top and three walls, each
                        point a small sphere (a stand-in for a depth-camera cloud);
* ``random_scene``      a random mix of spheres, capsules and boxes.

Primitive rows (FP32):
  spheres   [n][4]   centre, radius
  capsules  [n][7]   end point p0, end point p1, radius
  cylinders [n][8]   centre, unit axis, half height, radius
  boxes     [n][15]  centre, row-major 3x3 rotation (columns are the box axes), half extents

A keep-out rule redraws primitives whose bounding ball comes within 0.25 m of a robot mount
point; the redraws are part of the seeded stream.
"""
from __future__ import annotations

import numpy as np

KEEP_OUT = 0.25


def _rand_rotation(g: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    w, x, y, z = g.normal(size=4)
    n = np.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _clear_of(centre: np.ndarray, bound: float, mounts: np.ndarray) -> bool:
    dist = np.sqrt(((mounts - centre[None, :]) ** 2).sum(axis=1))
    return bool(np.all(dist >= KEEP_OUT + bound))


def _empty() -> dict:
    return {"spheres": np.zeros((0, 4), np.float32), "capsules": np.zeros((0, 7), np.float32),
            "cylinders": np.zeros((0, 8), np.float32), "boxes": np.zeros((0, 15), np.float32)}


def empty_scene() -> dict:
    return _empty()


def _pack(spheres=(), capsules=(), cylinders=(), boxes=()) -> dict:
    env = _empty()
    for key, rows, width in (("spheres", spheres, 4), ("capsules", capsules, 7),
                             ("cylinders", cylinders, 8), ("boxes", boxes, 15)):
        if len(rows):
            env[key] = np.asarray(rows, dtype=np.float64).reshape(-1, width).astype(np.float32)
    return env


def _sphere(g, mounts, rmin=0.05, rmax=0.2):
    while True:
        c = g.uniform(-1.0, 1.0, 3)
        r = g.uniform(rmin, rmax)
        if _clear_of(c, r, mounts):
            return np.concatenate([c, [r]])


def _box(g, mounts, emin=0.05, emax=0.3):
    while True:
        c = g.uniform(-1.0, 1.0, 3)
        e = g.uniform(emin, emax, 3)
        rot = _rand_rotation(g)
        if _clear_of(c, float(np.linalg.norm(e)), mounts):
            return np.concatenate([c, rot.reshape(-1), e])


def _capsule(g, mounts, hmin=0.05, hmax=0.3, rmin=0.02, rmax=0.1):
    while True:
        c = g.uniform(-1.0, 1.0, 3)
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        h = g.uniform(hmin, hmax)
        r = g.uniform(rmin, rmax)
        if _clear_of(c, h + r, mounts):
            return np.concatenate([c - h * u, c + h * u, [r]])


def cube_scene(g: np.random.Generator, n_spheres: int = 32, n_boxes: int = 8,
               mounts=((0.0, 0.0, 0.0),), sphere_r=(0.05, 0.2)) -> dict:
    """Random spheres (r ~ U[sphere_r]) and oriented boxes in the cube [-1, 1]^3."""
    m = np.asarray(mounts, dtype=np.float64).reshape(-1, 3)
    spheres = [_sphere(g, m, *sphere_r) for _ in range(n_spheres)]
    boxes = [_box(g, m) for _ in range(n_boxes)]
    return _pack(spheres=spheres, boxes=boxes)


def _box_clear(centre, rot, ext, mounts) -> bool:
    """Exact distance from every mount point to the oriented box is at least KEEP_OUT."""
    for p in mounts:
        local = rot.T @ (p - centre)
        if np.linalg.norm(np.maximum(np.abs(local) - ext, 0.0)) < KEEP_OUT:
            return False
    return True


def shelf_scene(g: np.random.Generator, n_units: int = 12, n_loose: int = 4,
                n_capsules: int = 50, mounts=((0.0, 0.0, 0.0),), radius=(1.0, 1.5),
                keepout: str = "unit") -> dict:
    """Shelf units in a half ring in front of the base (+x side): 8 boxes per unit (two side
    panels, a back panel, five boards), loose boxes and upright capsules standing on boards.

    Units stand at a radial distance U[radius].  keepout="unit" keeps each unit's bounding ball
    out of the mounts' keep-out balls (so units start about 1 m out); keepout="box" checks each
    panel, loose box and capsule on its own (exact box distance), which lets units stand closer
    (radius (0.55, 1.1) puts them in the arm's reach)."""
    m = np.asarray(mounts, dtype=np.float64).reshape(-1, 3)
    boxes, boards = [], []
    t = 0.01                                           # half thickness of every panel
    per_box = keepout == "box"
    for k in range(n_units):
        while True:
            yaw = np.pi * ((k + 0.5 + g.uniform(-0.3, 0.3)) / n_units - 0.5)
            rad = g.uniform(*radius)
            z0 = g.uniform(-0.3, 0.3)
            w = g.uniform(0.25, 0.4)                   # half width
            dep = g.uniform(0.15, 0.2)                 # half depth
            h = g.uniform(0.4, 0.7)                    # half height
            # unit frame: x points away from the base, y along the width, z up
            cy, sy = np.cos(yaw), np.sin(yaw)
            rot = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
            centre = np.array([rad * cy, rad * sy, z0 + h])
            bound = float(np.sqrt(dep * dep + w * w + h * h))
            parts = []
            for side in (-1.0, 1.0):                   # side panels
                parts.append((np.array([0.0, side * w, 0.0]), np.array([dep, t, h])))
            parts.append((np.array([dep, 0.0, 0.0]), np.array([t, w, h])))   # back panel
            for i in range(5):                         # boards, bottom to top
                z = -h + 2.0 * h * i / 4.0
                parts.append((np.array([0.0, 0.0, z]), np.array([dep, w, t])))
            if per_box:
                if all(_box_clear(centre + rot @ off, rot, ext, m) for off, ext in parts):
                    break
            elif _clear_of(centre, bound, m):
                break
        for i in range(5):
            z = -h + 2.0 * h * i / 4.0
            boards.append((centre + rot @ np.array([0.0, 0.0, z]), rot, dep, w))
        for off, ext in parts:
            boxes.append(np.concatenate([centre + rot @ off, rot.reshape(-1), ext]))
    for _ in range(n_loose):                           # small boxes lying on random boards
        while True:
            c, rot, dep, w = boards[g.integers(0, len(boards))]
            e = g.uniform(0.04, 0.1, 3)
            e[:2] = np.minimum(e[:2], [dep, w])
            x = g.uniform(-dep + e[0], dep - e[0])
            y = g.uniform(-w + e[1], w - e[1])
            bc = c + rot @ np.array([x, y, t + e[2]])
            if not per_box or _box_clear(bc, rot, e, m):
                break
        boxes.append(np.concatenate([bc, rot.reshape(-1), e]))
    capsules = []
    for _ in range(n_capsules):
        while True:
            c, rot, dep, w = boards[g.integers(0, len(boards))]
            r = g.uniform(0.02, 0.05)
            hl = g.uniform(0.04, 0.12)
            x = g.uniform(-dep + r, dep - r)
            y = g.uniform(-w + r, w - r)
            base = c + rot @ np.array([x, y, t + r])
            if not per_box or _clear_of(base + np.array([0.0, 0.0, hl]), hl + r, m):
                break
        capsules.append(np.concatenate([base, base + np.array([0.0, 0.0, 2.0 * hl]), [r]]))
    return _pack(capsules=capsules, boxes=boxes)


def point_cloud_scene(g: np.random.Generator, n_spheres: int = 300, n_points: int = 20000,
                      point_r: float = 0.01, mounts=((0.0, 0.0, 0.0),),
                      sphere_r=(0.01, 0.04)) -> dict:
    """Random spheres plus a noisy table top (z = 0.4) and three walls sampled as points."""
    m = np.asarray(mounts, dtype=np.float64).reshape(-1, 3)
    spheres = [_sphere(g, m, *sphere_r) for _ in range(n_spheres)]
    per = n_points // 4
    patches = []
    # (centre, u axis, v axis, normal) -- each patch 1.0-1.5 m per side, >= 0.4 m from the axis
    su, sv = g.uniform(1.0, 1.5, 4), g.uniform(1.0, 1.5, 4)
    patches.append((np.array([0.4 + su[0] / 2, 0.0, 0.4]), np.array([1.0, 0, 0]),
                    np.array([0, 1.0, 0]), np.array([0, 0, 1.0])))
    patches.append((np.array([1.2, 0.0, 0.4]), np.array([0, 1.0, 0]),
                    np.array([0, 0, 1.0]), np.array([1.0, 0, 0])))
    patches.append((np.array([0.2, 1.1, 0.4]), np.array([1.0, 0, 0]),
                    np.array([0, 0, 1.0]), np.array([0, 1.0, 0])))
    patches.append((np.array([0.2, -1.1, 0.4]), np.array([1.0, 0, 0]),
                    np.array([0, 0, 1.0]), np.array([0, 1.0, 0])))
    pts = []
    for k, (c, u, v, nrm) in enumerate(patches):
        a = g.uniform(-su[k] / 2, su[k] / 2, per)
        b = g.uniform(-sv[k] / 2, sv[k] / 2, per)
        e = g.normal(0.0, 0.005, per)
        pts.append(c[None, :] + a[:, None] * u + b[:, None] * v + e[:, None] * nrm)
    pts = np.concatenate(pts, axis=0)
    cloud = np.concatenate([pts, np.full((len(pts), 1), point_r)], axis=1)
    return _pack(spheres=np.concatenate([np.asarray(spheres).reshape(-1, 4), cloud], axis=0))


def random_scene(g: np.random.Generator, lo: int = 50, hi: int = 300,
                 mounts=((0.0, 0.0, 0.0),)) -> dict:
    """U{lo..hi} primitives, each a sphere, capsule or box with equal probability."""
    m = np.asarray(mounts, dtype=np.float64).reshape(-1, 3)
    n = int(g.integers(lo, hi + 1))
    kinds = g.integers(0, 3, n)
    spheres = [_sphere(g, m, 0.02, 0.1) for _ in range(int((kinds == 0).sum()))]
    capsules = [_capsule(g, m) for _ in range(int((kinds == 1).sum()))]
    boxes = [_box(g, m, 0.03, 0.15) for _ in range(int((kinds == 2).sum()))]
    return _pack(spheres=spheres, capsules=capsules, boxes=boxes)


def scene_summary(env: dict) -> dict:
    return {k: int(len(v)) for k, v in env.items()}
