"""Pins of the oracle's forward kinematics and sphere placement (Sec. III-B, III-C).

Nothing here re-types the oracle's DH product: the oracle is checked against hand-worked
values (tests/golden/fk_hand.json), a closed form for planar chains, a second formulation
(product of exponentials with Rodrigues rotations about the joint axes) and rigid-motion
invariants.
"""
import json
import os

import numpy as np
import pytest

from synthetic import chain_robot, bimanual_robot, lift_arm_robot, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _robot_from_case(case):
    dh = np.asarray(case["dh"], dtype=np.float64)
    dof = len(dh)
    spheres = np.asarray(case.get("spheres", []), dtype=np.float64).reshape(-1, 5)
    return {
        "dof": dof,
        "parent_link": np.asarray(case.get("parent_link", list(range(dof))), dtype=np.int32),
        "mount": np.asarray(case["mount"], dtype=np.float64) if "mount" in case else None,
        "dh": dh,
        "sphere_link": spheres[:, 0].astype(np.int32),
        "sphere_xyzr": spheres[:, 1:5],
        "self_pairs": np.zeros((0, 2), np.int32),
        "joint_type": np.asarray(case["joint_type"], np.int32) if "joint_type" in case else None,
    }


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "fk_hand.json")))["cases"],
                         ids=lambda c: c["name"])
def test_fk_hand_values(orc, case):
    robot = _robot_from_case(case)
    T, _ = orc.fk(robot, case["q"])
    if "link_origins" in case:
        np.testing.assert_allclose(T[:, :, 3], np.asarray(case["link_origins"]), atol=1e-12)
    if "centres" in case:
        c = orc.sphere_centres(robot, case["q"])
        np.testing.assert_allclose(c, np.asarray(case["centres"]), atol=1e-12)


def test_planar_closed_form(orc):
    """alpha = 0 chains: x = sum a_i cos(sum_{k<=i} q_k), y = same with sin, z = sum d_i."""
    g = np.random.default_rng(1)
    for dof in (1, 2, 3, 5, 9):
        a = g.uniform(0.1, 1.0, dof)
        d = g.uniform(0.0, 0.5, dof)
        dh = np.stack([a, d, np.ones(dof), np.zeros(dof), g.uniform(-1, 1, dof)], axis=1)
        robot = _robot_from_case({"dh": dh.tolist()})
        for _ in range(20):
            q = g.uniform(-3.0, 3.0, dof)
            T, _ = orc.fk(robot, q)
            ang = np.cumsum(q + dh[:, 4])
            exp = np.array([np.sum(a * np.cos(ang)), np.sum(a * np.sin(ang)), np.sum(d)])
            np.testing.assert_allclose(T[-1, :, 3], exp, atol=1e-12)


def test_mount_under_a_moving_parent(orc):
    """A fixed mount sits between the parent link and the joint (T_parent M A): a planar 2R
    chain with unit links whose second joint is mounted 0.5 along link 1's x axis and turned a
    quarter turn about z.  Closed form: link 2's origin is 1.5 (cos q1, sin q1) plus the unit
    vector at angle q1 + pi/2 + q2, which is also the direction of link 2's x axis."""
    phi, m = np.pi / 2, 0.5
    mount = [[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0],
             [np.cos(phi), -np.sin(phi), 0, m, np.sin(phi), np.cos(phi), 0, 0, 0, 0, 1, 0]]
    robot = _robot_from_case({"dh": [[1, 0, 1, 0, 0], [1, 0, 1, 0, 0]], "mount": mount})
    g = np.random.default_rng(4)
    for _ in range(20):
        q1, q2 = g.uniform(-3.0, 3.0, 2)
        T, _ = orc.fk(robot, [q1, q2])
        th = q1 + phi + q2
        want = [1.5 * np.cos(q1) + np.cos(th), 1.5 * np.sin(q1) + np.sin(th), 0.0]
        np.testing.assert_allclose(T[2, :, 3], want, atol=1e-12)
        np.testing.assert_allclose(T[2, :, 0], [np.cos(th), np.sin(th), 0.0], atol=1e-12)


def _rodrigues(axis, angle):
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * k + (1 - np.cos(angle)) * k @ k


@pytest.mark.parametrize("kind", ["chain7", "chain8", "bimanual", "lift"])
def test_product_of_exponentials(orc, kind):
    """A second formulation: T_link(q) = prod_{j in path} exp(xi_j q_j) * T_link(0), with the
    twists xi_j taken from the joint axes and points at the zero pose: a rotation about the
    axis through the point for a revolute joint, a translation along the axis for a prismatic
    one."""
    g = rng("pins", kind)
    robot = {"chain7": lambda: chain_robot(g, 7, 2), "chain8": lambda: chain_robot(g, 8, 2, 2),
             "bimanual": lambda: bimanual_robot(g, 3, 2, 2),
             "lift": lambda: lift_arm_robot(g, 4, 2, 2)}[kind]()
    jt = robot.get("joint_type")
    jt = np.zeros(robot["dof"], int) if jt is None else jt
    dof = robot["dof"]
    T0, P0 = orc.fk(robot, np.zeros(dof))
    parent = np.concatenate([[-1], robot["parent_link"]])
    for _ in range(10):
        q = g.uniform(-2.9, 2.9, dof)
        T, _ = orc.fk(robot, q)
        for link in range(1, dof + 1):
            path = []
            k = link
            while k > 0:
                path.append(k - 1)
                k = parent[k]
            M = np.eye(4)
            for j in reversed(path):       # base-most joint first
                E = np.eye(4)
                if jt[j] == 1:
                    E[:3, 3] = P0[j][:, 2] * q[j]
                else:
                    R = _rodrigues(P0[j][:, 2], q[j])
                    o = P0[j][:, 3]
                    E[:3, :3] = R
                    E[:3, 3] = o - R @ o
                M = M @ E
            Tz = np.eye(4)
            Tz[:3, :] = T0[link]
            np.testing.assert_allclose((M @ Tz)[:3, :], T[link], atol=1e-12)


@pytest.mark.parametrize("kind", ["chain7", "bimanual"])
def test_rigid_invariants(orc, kind):
    g = rng("pins", "rigid" + kind)
    robot = chain_robot(g, 7, 6) if kind == "chain7" else bimanual_robot(g, 7, 8, 8)
    dh = robot["dh"].astype(np.float64)
    xyzr = robot["sphere_xyzr"].astype(np.float64)
    sl = robot["sphere_link"]
    for _ in range(20):
        q = g.uniform(-2.9, 2.9, robot["dof"])
        T, P = orc.fk(robot, q)
        R = T[:, :, :3]
        for k in range(len(T)):
            np.testing.assert_allclose(R[k].T @ R[k], np.eye(3), atol=1e-12)
            assert abs(np.linalg.det(R[k]) - 1.0) < 1e-12
        # each joint frame origin to its link origin spans the DH link length hypot(a, d)
        for j in range(robot["dof"]):
            dist = np.linalg.norm(T[j + 1][:, 3] - P[j][:, 3])
            assert abs(dist - np.hypot(dh[j, 0], dh[j, 1])) < 1e-12
        c = orc.sphere_centres(robot, q)
        dist = np.linalg.norm(c - T[sl][:, :, 3], axis=1)
        np.testing.assert_allclose(dist, np.linalg.norm(xyzr[:, :3], axis=1), atol=1e-12)


def test_joint_moves_only_descendants(orc):
    """Joint j of one arm leaves the spheres of the other arm and the torso in place."""
    g = rng("pins", "tree")
    robot = bimanual_robot(g, 7, 8, 8)
    q = g.uniform(-2.9, 2.9, 14)
    c0 = orc.sphere_centres(robot, q)
    q2 = q.copy()
    q2[3] += 0.5                                       # left arm, joint 3 -> moves links 4..7
    c1 = orc.sphere_centres(robot, q2)
    moved = np.linalg.norm(c1 - c0, axis=1) > 1e-9
    sl = robot["sphere_link"]
    assert not moved[(sl <= 3) | (sl >= 8)].any()
    assert moved[(sl >= 5) & (sl <= 7)].any()
