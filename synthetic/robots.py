"""Seeded synthetic robots: revolute DH chains with collision spheres per link.

The method models a robot as a kinematic tree whose links carry collision spheres
(Sec. III-C, "Vectorized Collision Checking"); the evaluation uses a 7-DoF arm, an 8-DoF
mobile manipulator and a 14-DoF two-armed robot (Sec. IV).  The robots here are synthetic
stand-ins of those sizes:

* joints are revolute with standard DH parameters; a ~ U[0, 0.1] m, d ~ U[0, 0.4] m, the twist
  is drawn from {-pi/2, 0, +pi/2} and stored as its exact (cos, sin) pair, limits are +-2.9 rad;
* the spheres of link j lie along the segment from the previous joint origin to frame j's
  origin; in frame j that previous origin is the constant vector (-a, -d sin(alpha),
  -d cos(alpha)) of the DH parameters, so the sphere layout is configuration independent;
* each joint's (a, d) is redrawn until the link segment hypot(a, d) is at least 0.15 m, so
  that spheres on links two apart are not permanently in contact (a short middle link would
  fold them onto each other and make every configuration self-colliding);
* the self-collision pair list holds every sphere pair on links that are neither equal nor
  joined by a joint (the base or torso is link 0; two arms on one torso are never adjacent),
  optionally cut to a requested size by a seeded subsample without replacement.

Arrays are canonical FP32 (int32 for indices); everything is drawn from the workload rng.
"""
from __future__ import annotations

import numpy as np

# exact (cos, sin) of the three twist values
_TWIST = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0]], dtype=np.float64)
Q_LIMIT = 2.9


def _identity_mount() -> np.ndarray:
    m = np.zeros(12, dtype=np.float64)
    m[0] = m[5] = m[10] = 1.0
    return m


def _mount(tx: float, ty: float, tz: float, rx_cos: float, rx_sin: float) -> np.ndarray:
    """Row-major 3x4 of a translation followed by a rotation about x (exact cos/sin)."""
    return np.array([1.0, 0.0, 0.0, tx,
                     0.0, rx_cos, -rx_sin, ty,
                     0.0, rx_sin, rx_cos, tz], dtype=np.float64)


MIN_LINK = 0.15


def _draw_joints(g: np.random.Generator, n: int) -> np.ndarray:
    """a ~ U[0, 0.1], d ~ U[0, 0.4], redrawn until hypot(a, d) >= MIN_LINK; twist code."""
    dh = np.zeros((n, 5), dtype=np.float64)
    for j in range(n):
        while True:
            a = g.uniform(0.0, 0.1)
            d = g.uniform(0.0, 0.4)
            if np.hypot(a, d) >= MIN_LINK:
                break
        k = g.integers(0, 3)
        dh[j, 0], dh[j, 1] = a, d
        dh[j, 2], dh[j, 3] = _TWIST[k, 0], _TWIST[k, 1]
    return dh


def _link_spheres(g: np.random.Generator, dh_row: np.ndarray, n: int,
                  rmin: float = 0.03, rmax: float = 0.08) -> np.ndarray:
    """Spheres along the link segment, in the link's own frame."""
    a, d, ca, sa = dh_row[0], dh_row[1], dh_row[2], dh_row[3]
    v = np.array([-a, -d * sa, -d * ca])          # previous joint origin seen from frame j
    t = (np.arange(n) + 0.5) / n
    xyz = t[:, None] * v[None, :] + g.uniform(-0.02, 0.02, (n, 3))
    r = g.uniform(rmin, rmax, n)
    return np.concatenate([xyz, r[:, None]], axis=1)


def link_parents(parent_link: np.ndarray) -> np.ndarray:
    """parent[k] of every link k (link 0 is the fixed base and has parent -1)."""
    dof = len(parent_link)
    par = np.full(dof + 1, -1, dtype=np.int64)
    par[1:] = parent_link
    return par


def candidate_pairs(parent_link: np.ndarray, sphere_link: np.ndarray) -> np.ndarray:
    """All sphere pairs (s, t), s < t, on links that are neither equal nor adjacent."""
    par = link_parents(parent_link)
    sl = np.asarray(sphere_link)
    s_idx, t_idx = np.triu_indices(len(sl), k=1)
    la, lb = sl[s_idx], sl[t_idx]
    keep = (la != lb) & (par[lb] != la) & (par[la] != lb)
    return np.stack([s_idx[keep], t_idx[keep]], axis=1).astype(np.int64)


def _finish(dof, parent_link, mount, dh, sphere_link, xyzr, n_per_link, n_pairs, g):
    pairs = candidate_pairs(parent_link, sphere_link)
    if n_pairs is not None and n_pairs < len(pairs):
        pick = np.sort(g.choice(len(pairs), size=n_pairs, replace=False))
        pairs = pairs[pick]
    return {
        "dof": int(dof),
        "parent_link": np.asarray(parent_link, dtype=np.int32),
        "mount": np.asarray(mount, dtype=np.float32).reshape(dof, 12),
        "dh": np.asarray(dh, dtype=np.float32),
        "q_lo": np.full(dof, -Q_LIMIT, dtype=np.float32),
        "q_hi": np.full(dof, Q_LIMIT, dtype=np.float32),
        "sphere_link": np.asarray(sphere_link, dtype=np.int32),
        "sphere_xyzr": np.asarray(xyzr, dtype=np.float32),
        "self_pairs": np.asarray(pairs, dtype=np.int32).reshape(-1, 2),
    }


def chain_robot(g: np.random.Generator, dof: int, spheres_per_link: int,
                base_spheres: int = 0, n_pairs: int | None = None) -> dict:
    """Serial revolute chain; link 0 is the fixed base (optionally with spheres on -z)."""
    dh = _draw_joints(g, dof)
    parent_link = np.arange(dof)
    mount = np.tile(_identity_mount(), (dof, 1))
    rows, links, counts = [], [], [base_spheres]
    if base_spheres:
        z = -0.1 * np.arange(1, base_spheres + 1)
        r = g.uniform(0.03, 0.08, base_spheres)
        rows.append(np.stack([np.zeros_like(z), np.zeros_like(z), z, r], axis=1))
        links += [0] * base_spheres
    for j in range(dof):
        rows.append(_link_spheres(g, dh[j], spheres_per_link))
        links += [j + 1] * spheres_per_link
        counts.append(spheres_per_link)
    xyzr = np.concatenate(rows, axis=0)
    return _finish(dof, parent_link, mount, dh, np.array(links), xyzr, np.array(counts),
                   n_pairs, g)


LIFT_RANGE = (0.0, 0.4)


def lift_arm_robot(g: np.random.Generator, arm_dof: int = 7, spheres_per_link: int = 6,
                   torso_spheres: int = 4, n_pairs: int | None = None) -> dict:
    """A mobile-manipulator-like tree: joint 0 is a prismatic lift along the base z axis
    (stroke LIFT_RANGE, frame 0.3 m up at zero stroke) carrying a torso column (link 1,
    spheres below the lift frame) and a revolute arm on top of it (joints 1..arm_dof)."""
    dof = arm_dof + 1
    dh = np.concatenate([np.array([[0.0, 0.3, 1.0, 0.0, 0.0]]), _draw_joints(g, arm_dof)], axis=0)
    parent_link = np.arange(dof)
    mount = np.tile(_identity_mount(), (dof, 1))
    z = -0.1 * np.arange(0, torso_spheres)
    r = g.uniform(0.05, 0.08, torso_spheres)
    rows = [np.stack([np.zeros_like(z), np.zeros_like(z), z, r], axis=1)]
    links = [1] * torso_spheres
    counts = [0, torso_spheres]
    for j in range(1, dof):
        rows.append(_link_spheres(g, dh[j], spheres_per_link))
        links += [j + 1] * spheres_per_link
        counts.append(spheres_per_link)
    xyzr = np.concatenate(rows, axis=0)
    robot = _finish(dof, parent_link, mount, dh, np.array(links), xyzr, np.array(counts),
                    n_pairs, g)
    robot["joint_type"] = np.array([1] + [0] * arm_dof, dtype=np.int32)
    robot["q_lo"][0], robot["q_hi"][0] = LIFT_RANGE
    return robot


def bimanual_robot(g: np.random.Generator, arm_dof: int = 7, spheres_per_link: int = 8,
                   torso_spheres: int = 8, n_pairs: int | None = None) -> dict:
    """Two serial arms mounted left and right on a fixed torso (link 0)."""
    dof = 2 * arm_dof
    dh = np.concatenate([_draw_joints(g, arm_dof), _draw_joints(g, arm_dof)], axis=0)
    parent_link = np.concatenate([np.arange(arm_dof), np.arange(arm_dof) + arm_dof])
    parent_link[arm_dof] = 0
    mount = np.tile(_identity_mount(), (dof, 1))
    mount[0] = _mount(0.0, 0.25, 0.5, 0.0, -1.0)         # Rx(-pi/2): joint axis along +y
    mount[arm_dof] = _mount(0.0, -0.25, 0.5, 0.0, 1.0)   # Rx(+pi/2): joint axis along -y
    z = 0.1 * np.arange(1, torso_spheres + 1)
    r = g.uniform(0.03, 0.08, torso_spheres)
    rows = [np.stack([np.zeros_like(z), np.zeros_like(z), z, r], axis=1)]
    links = [0] * torso_spheres
    counts = [torso_spheres]
    for j in range(dof):
        rows.append(_link_spheres(g, dh[j], spheres_per_link))
        links += [j + 1] * spheres_per_link
        counts.append(spheres_per_link)
    xyzr = np.concatenate(rows, axis=0)
    return _finish(dof, parent_link, mount, dh, np.array(links), xyzr, np.array(counts),
                   n_pairs, g)


def robot_summary(robot: dict) -> dict:
    return {"dof": robot["dof"], "spheres": int(len(robot["sphere_link"])),
            "self_pairs": int(len(robot["self_pairs"]))}
