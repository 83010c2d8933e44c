"""Pins of the oracle's squared-penetration cost and its gradient.

A hand-worked one-link case, FP64 central differences of the cost (h = 1e-6), the geometric
Jacobian column checked against differences of the sphere centres, and a symmetry that forces
one gradient component to zero.
"""
import numpy as np
import pytest

from synthetic import workload, chain_robot, lift_arm_robot, rng, empty_scene


def _one_link():
    return {"dof": 1, "parent_link": np.array([0], np.int32), "mount": None,
            "dh": np.array([[1.0, 0.0, 1.0, 0.0, 0.0]]),
            "sphere_link": np.array([1], np.int32), "sphere_xyzr": np.array([[0, 0, 0, 0.1]]),
            "self_pairs": np.zeros((0, 2), np.int32)}


def test_hand_value(orc):
    """Sphere r = 0.1 at (cos q, sin q, 0); obstacle r = 0.1 at (1, 0.1, 0).  At q = 0 the
    centres are 0.1 apart: penetration 0.1, cost 0.01, and dC/dq = 2 * 0.1 * 1 = 0.2 (the
    distance shrinks at unit rate as the sphere turns towards +y)."""
    env = {"spheres": np.array([[1.0, 0.1, 0.0, 0.1]])}
    assert abs(orc.cost(_one_link(), env, [0.0]) - 0.01) < 1e-15
    assert abs(orc.cost_grad(_one_link(), env, [0.0])[0] - 0.2) < 1e-12


def test_zero_cost_iff_no_penetration(orc):
    w = workload("cost7", n=8)
    rb, ev = orc.Robot(w["robot"]), orc.Env(w["env"])
    cost = orc.costs(rb, ev, w["q"])
    cmin, _ = orc.states(rb, ev, w["q"])
    assert np.all((cost == 0.0) == (cmin >= 0.0))
    assert (cost > 0).any() and (cost == 0).any()
    g = orc.cost_grads(rb, ev, w["q"])
    assert np.all(g[:, cost == 0.0] == 0.0)


def _fd_case(orc, name, n, tol):
    w = workload(name, n=n)
    rb, ev = orc.Robot(w["robot"]), orc.Env(w["env"])
    q = w["q"].astype(np.float64)
    checked = 0
    for i in range(q.shape[1]):
        if orc.cost(rb, ev, q[:, i]) == 0.0:
            continue
        ga = orc.cost_grad(rb, ev, q[:, i])
        gf = orc.cost_grad_fd(rb, ev, q[:, i], h=1e-6)
        assert np.linalg.norm(ga - gf) <= tol * max(np.linalg.norm(ga), 1e-3), (i, ga, gf)
        checked += 1
    assert checked > 10


def test_gradient_matches_central_differences(orc):
    _fd_case(orc, "cost7", 96, 1e-6)


def test_gradient_all_primitive_kinds(orc):
    """Capsules and cylinders are absent from the cost workload; add them explicitly."""
    g = rng("pins", "grad-kinds")
    robot = chain_robot(g, 7, 6)
    env = {"capsules": np.array([[0.3, 0.2, 0.1, 0.5, -0.3, 0.6, 0.15],
                                 [-0.4, 0.1, 0.3, -0.2, 0.4, 0.5, 0.1]]),
           "cylinders": np.array([[0.2, -0.3, 0.4, 0.0, 0.6, 0.8, 0.3, 0.2],
                                  [-0.3, -0.2, 0.2, 1.0, 0.0, 0.0, 0.25, 0.15]]),
           "boxes": np.array([[0.1, 0.4, 0.3, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.2, 0.1, 0.3]])}
    rb, ev = orc.Robot(robot), orc.Env(env)
    checked = 0
    for _ in range(200):
        q = g.uniform(-2.9, 2.9, 7)
        if orc.cost(rb, ev, q) == 0.0:
            continue
        ga = orc.cost_grad(rb, ev, q)
        gf = orc.cost_grad_fd(rb, ev, q)
        assert np.linalg.norm(ga - gf) <= 1e-6 * max(np.linalg.norm(ga), 1e-3)
        checked += 1
    assert checked > 20


def test_self_only_first_joint_is_free(orc):
    """With no base spheres and no obstacles, turning the whole chain about the first joint's
    axis keeps every self distance: dC/dq_0 = 0."""
    w = workload("cost7", n=64)
    rb, ev = orc.Robot(w["robot"]), orc.Env(empty_scene())
    q = w["q"].astype(np.float64)
    hits = 0
    for i in range(q.shape[1]):
        if orc.cost(rb, ev, q[:, i]) > 0:
            g = orc.cost_grad(rb, ev, q[:, i])
            assert abs(g[0]) <= 1e-12 * max(1.0, np.abs(g).max())
            hits += 1
    assert hits > 0


def test_jacobian_column_matches_centre_differences(orc):
    """d c_s / d q_j = z_j x (c_s - o_j) for spheres moved by joint j, else 0."""
    g = rng("pins", "jac")
    robot = chain_robot(g, 7, 3)
    rb = orc.Robot(robot)
    par = np.concatenate([[-1], robot["parent_link"]])
    for _ in range(5):
        q = g.uniform(-2.9, 2.9, 7)
        _, P = orc.fk(rb, q)
        c = orc.sphere_centres(rb, q)
        for j in range(7):
            h = 1e-6
            qp, qm = q.copy(), q.copy()
            qp[j] += h
            qm[j] -= h
            dc = (orc.sphere_centres(rb, qp) - orc.sphere_centres(rb, qm)) / (2 * h)
            for s, lk in enumerate(robot["sphere_link"]):
                k, moved = lk, False
                while k > 0:
                    moved |= (k == j + 1)
                    k = par[k]
                exp = np.cross(P[j][:, 2], c[s] - P[j][:, 3]) if moved else np.zeros(3)
                np.testing.assert_allclose(dc[s], exp, atol=1e-8)


def test_non_finite_cost(orc):
    assert np.isnan(orc.cost(_one_link(), {}, [np.nan]))
    assert np.isnan(orc.cost_grad(_one_link(), {}, [np.inf])).all()


def test_prismatic_gradient_and_jacobian(orc):
    """A prismatic lift: its Jacobian column is the slide axis itself (every sphere above it
    moves with unit speed along the axis), and the analytic gradient matches central
    differences of the cost."""
    g = rng("pins", "lift")
    robot = lift_arm_robot(g, 4, 3, 3)
    env = {"boxes": np.array([[0.2, 0.1, 0.45, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.25, 0.2, 0.1]]),
           "spheres": np.array([[0.0, 0.2, 0.6, 0.2]])}
    rb, ev = orc.Robot(robot), orc.Env(env)
    lo, hi = robot["q_lo"].astype(np.float64), robot["q_hi"].astype(np.float64)
    checked = 0
    for _ in range(300):
        q = g.uniform(lo, hi)
        _, P = orc.fk(rb, q)
        h = 1e-6
        qp, qm = q.copy(), q.copy()
        qp[0] += h
        qm[0] -= h
        dc = (orc.sphere_centres(rb, qp) - orc.sphere_centres(rb, qm)) / (2 * h)
        np.testing.assert_allclose(dc, np.tile(P[0][:, 2], (len(dc), 1)), atol=1e-8)
        if orc.cost(rb, ev, q) == 0.0:
            continue
        ga = orc.cost_grad(rb, ev, q)
        gf = orc.cost_grad_fd(rb, ev, q)
        assert np.linalg.norm(ga - gf) <= 1e-6 * max(np.linalg.norm(ga), 1e-3)
        checked += 1
    assert checked > 20
