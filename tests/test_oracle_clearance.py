"""Pins of the oracle's signed distances to the primitive types (Sec. III-C).

Hand-worked values (tests/golden/clearance_hand.json), special cases that reduce to another
shape, brute-force sampling of each primitive's surface, an independent inside/outside test
and invariance under a rigid motion of shape and point together.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HAND = json.load(open(os.path.join(GOLDEN, "clearance_hand.json")))


@pytest.mark.parametrize("case", HAND["cases"], ids=lambda c: c["kind"] + ":" + str(c["point"]))
def test_hand_values(orc, case):
    kind = HAND["kinds"][case["kind"]]
    assert abs(orc.sd(kind, case["point"], case["prim"]) - case["sd"]) < 1e-12
    # clearance of a robot sphere is the point's signed distance minus its radius
    assert abs(orc.clearance(kind, case["point"], 0.07, case["prim"]) - (case["sd"] - 0.07)) < 1e-12


def _rot(g):
    q = g.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _random_prims(g):
    c = g.uniform(-1, 1, 3)
    R = _rot(g)
    e = g.uniform(0.1, 0.6, 3)
    box = np.concatenate([c, R.reshape(-1), e])
    p0 = g.uniform(-1, 1, 3)
    p1 = p0 + g.uniform(-0.8, 0.8, 3)
    cap = np.concatenate([p0, p1, [g.uniform(0.1, 0.4)]])
    w = g.normal(size=3)
    w /= np.linalg.norm(w)
    cyl = np.concatenate([c, w, [g.uniform(0.1, 0.6), g.uniform(0.1, 0.5)]])
    sph = np.concatenate([c, [g.uniform(0.1, 0.5)]])
    return {0: sph, 1: cap, 2: cyl, 3: box}


def _surface_samples(kind, prim, n=160):
    """Dense samples of the primitive's boundary, written from each shape's parametrisation."""
    u = (np.arange(n) + 0.5) / n
    if kind == 0:
        th, ph = np.meshgrid(np.pi * u, 2 * np.pi * u, indexing="ij")
        d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1).reshape(-1, 3)
        return prim[:3] + prim[3] * d
    if kind == 3:
        c, R, e = prim[:3], prim[3:12].reshape(3, 3), prim[12:15]
        s = np.linspace(-1, 1, n)
        a, b = np.meshgrid(s, s, indexing="ij")
        pts = []
        for ax in range(3):
            o1, o2 = [k for k in range(3) if k != ax]
            for sign in (-1.0, 1.0):
                p = np.zeros((a.size, 3))
                p[:, ax] = sign * e[ax]
                p[:, o1] = a.ravel() * e[o1]
                p[:, o2] = b.ravel() * e[o2]
                pts.append(p)
        return c + np.concatenate(pts) @ R.T
    # capsule and cylinder: build a frame around the axis
    if kind == 1:
        p0, p1, r = prim[:3], prim[3:6], prim[6]
        axis = p1 - p0
        L = np.linalg.norm(axis)
        w = axis / L
    else:
        o, w, H, r = prim[:3], prim[3:6], prim[6], prim[7]
        p0, L = o - H * w, 2 * H
    t1 = np.cross(w, [1.0, 0, 0] if abs(w[0]) < 0.9 else [0, 1.0, 0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(w, t1)
    ph = 2 * np.pi * u
    ring = np.cos(ph)[:, None] * t1 + np.sin(ph)[:, None] * t2
    hs = np.linspace(0, L, n)
    side = (p0 + hs[:, None, None] * w + r * ring[None]).reshape(-1, 3)
    if kind == 1:
        th = 0.5 * np.pi * u
        caps = []
        for end, sgn in ((p0, -1.0), (p0 + L * w, 1.0)):
            caps.append((end + r * (np.cos(th)[:, None, None] * ring[None]
                                    + sgn * np.sin(th)[:, None, None] * w)).reshape(-1, 3))
        return np.concatenate([side] + caps)
    rr = np.linspace(0, r, n)
    disc = (rr[:, None, None] * ring[None]).reshape(-1, 3)
    return np.concatenate([side, p0 + disc, p0 + L * w + disc])


def _inside(kind, prim, p):
    """Independent membership test (no distance formula)."""
    if kind == 0:
        return np.sum((p - prim[:3]) ** 2) < prim[3] ** 2
    if kind == 3:
        loc = prim[3:12].reshape(3, 3).T @ (p - prim[:3])
        return bool(np.all(np.abs(loc) < prim[12:15]))
    if kind == 1:
        # inside iff the distance to one of many points of the segment is below the radius
        ts = np.linspace(0, 1, 20001)
        seg = prim[:3] + ts[:, None] * (prim[3:6] - prim[:3])
        return bool(np.min(np.sum((seg - p) ** 2, axis=1)) < prim[6] ** 2)
    o, w, H, r = prim[:3], prim[3:6], prim[6], prim[7]
    h = np.dot(p - o, w)
    return abs(h) < H and np.linalg.norm(p - o - h * w) < r


@pytest.mark.parametrize("kind", [0, 1, 2, 3], ids=["sphere", "capsule", "cylinder", "box"])
def test_brute_force_surface(orc, kind):
    """|sd| equals the distance to the sampled boundary (within the sample spacing) and its
    sign agrees with an independent inside test."""
    g = np.random.default_rng(100 + kind)
    for _ in range(6):
        prim = _random_prims(g)[kind]
        surf = _surface_samples(kind, prim)
        spacing = 0.05          # generous bound on the sample spacing of every parametrisation
        for _ in range(25):
            p = prim[:3] + g.uniform(-1.2, 1.2, 3)
            sd = orc.sd(kind, p, prim)
            dmin = np.min(np.linalg.norm(surf - p, axis=1))
            assert dmin >= abs(sd) - 1e-9
            assert dmin - abs(sd) <= spacing
            if abs(sd) > 1e-3:
                assert (sd < 0) == _inside(kind, prim, p)


def test_degenerate_capsule_is_sphere(orc):
    g = np.random.default_rng(7)
    for _ in range(50):
        c = g.uniform(-1, 1, 3)
        r = g.uniform(0.05, 0.5)
        p = g.uniform(-2, 2, 3)
        cap = np.concatenate([c, c, [r]])
        assert abs(orc.sd(1, p, cap) - orc.sd(0, p, np.concatenate([c, [r]]))) < 1e-12


def test_rigid_motion_invariance(orc):
    g = np.random.default_rng(8)
    for _ in range(30):
        prims = _random_prims(g)
        R = _rot(g)
        t = g.uniform(-1, 1, 3)
        p = g.uniform(-1.5, 1.5, 3)
        mv = lambda x: R @ x + t
        box = prims[3]
        box2 = np.concatenate([mv(box[:3]), (R @ box[3:12].reshape(3, 3)).reshape(-1), box[12:]])
        cap = prims[1]
        cap2 = np.concatenate([mv(cap[:3]), mv(cap[3:6]), cap[6:]])
        cyl = prims[2]
        cyl2 = np.concatenate([mv(cyl[:3]), R @ cyl[3:6], cyl[6:]])
        for k, a, b in ((3, box, box2), (1, cap, cap2), (2, cyl, cyl2)):
            assert abs(orc.sd(k, p, a) - orc.sd(k, mv(p), b)) < 1e-12
