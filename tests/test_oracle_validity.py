"""Pins of the oracle's state and edge validity (Sec. III-C, III-D).

Hand-built robots with known answers, special cases, the edge discretization's hand counts and
the edge result re-derived through a second oracle path (materialised states).
"""
import numpy as np
import pytest

from synthetic import workload

INF = float("inf")


def _one_link(a=1.0, spheres=((0.0, 0.0, 0.0, 0.1),)):
    sp = np.asarray(spheres, dtype=np.float64)
    return {"dof": 1, "parent_link": np.array([0], np.int32), "mount": None,
            "dh": np.array([[a, 0.0, 1.0, 0.0, 0.0]]),
            "sphere_link": np.ones(len(sp), np.int32), "sphere_xyzr": sp,
            "self_pairs": np.zeros((0, 2), np.int32)}


def _env(spheres=(), capsules=(), cylinders=(), boxes=()):
    return {"spheres": np.asarray(spheres, float).reshape(-1, 4),
            "capsules": np.asarray(capsules, float).reshape(-1, 7),
            "cylinders": np.asarray(cylinders, float).reshape(-1, 8),
            "boxes": np.asarray(boxes, float).reshape(-1, 15)}


def test_nothing_to_test_is_free(orc):
    r = _one_link()
    assert orc.state_min_clearance(r, _env(), [0.3]) == INF
    assert orc.state_collides(r, _env(), [0.3]) == 0


def test_one_link_hand_values(orc):
    # sphere of radius 0.1 at the link origin, which sits at (cos q, sin q, 0)
    r = _one_link()
    env = _env(spheres=[[1.0, 0.0, 0.3, 0.1]])
    assert abs(orc.state_min_clearance(r, env, [0.0]) - 0.1) < 1e-12
    assert orc.state_collides(r, env, [0.0]) == 0
    env = _env(spheres=[[1.0, 0.0, 0.15, 0.1]])
    assert abs(orc.state_min_clearance(r, env, [0.0]) + 0.05) < 1e-12
    assert orc.state_collides(r, env, [0.0]) == 1
    # an axis-aligned box whose face is 0.25 from the sphere centre at q = pi/2 -> (0, 1, 0)
    box = [0.0, 1.5, 0.0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.5, 0.25, 0.5]
    assert abs(orc.state_min_clearance(r, _env(boxes=[box]), [np.pi / 2]) - 0.15) < 1e-12


def test_touching_is_free(orc):
    """A state collides only when some clearance is strictly negative.  The link origin sits at
    exactly (1, 0, 0) for q = 0, so a 0.25 sphere there touches a 0.75 sphere about the world
    origin with clearance exactly 0.0: free, as a state, in a batch and as a zero-length edge.
    Moved 1e-9 closer, it collides."""
    r = _one_link(spheres=((0.0, 0.0, 0.0, 0.25),))
    env = _env(spheres=[[0.0, 0.0, 0.0, 0.75]])
    assert orc.state_min_clearance(r, env, [0.0]) == 0.0
    assert orc.state_collides(r, env, [0.0]) == 0
    cmin, flag = orc.states(r, env, np.zeros((1, 3)))
    assert np.all(cmin == 0.0) and not flag.any()
    flag, _, emin = orc.edges(r, env, np.zeros((1, 1)), np.zeros((1, 1)), res=1.0 / 32.0)
    assert flag[0] == 0 and emin[0] == 0.0
    closer = _env(spheres=[[1e-9, 0.0, 0.0, 0.75]])
    assert orc.state_collides(r, closer, [0.0]) == 1
    assert orc.states(r, closer, np.zeros((1, 3)))[1].all()
    assert orc.edges(r, closer, np.zeros((1, 1)), np.zeros((1, 1)), res=1.0 / 32.0)[0][0] == 1


def test_self_pair_hand_value(orc):
    """Planar 3R with unit links at (0, 120, 120) deg closes an equilateral triangle: the
    origins of links 1 and 3 are 1 apart, so two 0.6 spheres there overlap by 0.2."""
    robot = {"dof": 3, "parent_link": np.arange(3, dtype=np.int32), "mount": None,
             "dh": np.array([[1.0, 0, 1, 0, 0]] * 3),
             "sphere_link": np.array([1, 3], np.int32),
             "sphere_xyzr": np.array([[0, 0, 0, 0.6], [0, 0, 0, 0.6]]),
             "self_pairs": np.array([[0, 1]], np.int32)}
    q = [0.0, 2 * np.pi / 3, 2 * np.pi / 3]
    assert abs(orc.state_min_clearance(robot, _env(), q) + 0.2) < 1e-12
    assert orc.state_collides(robot, _env(), q) == 1
    # straight chain: origins 2 apart -> clearance 0.8
    assert abs(orc.state_min_clearance(robot, _env(), [0, 0, 0]) - 0.8) < 1e-12


def test_non_finite_is_colliding(orc):
    r = _one_link()
    for bad in (np.nan, np.inf, -np.inf):
        assert orc.state_collides(r, _env(), [bad]) == 1
        assert np.isnan(orc.state_min_clearance(r, _env(), [bad]))


def test_sphere_on_robot_sphere_collides(orc):
    """An obstacle sphere centred on a robot sphere always overlaps it: clearance -(r + R)."""
    w = workload("states7", n=8)
    rb = orc.Robot(w["robot"])
    for i in range(8):
        q = w["q"][:, i].astype(np.float64)
        c = orc.sphere_centres(rb, q)
        s = 11
        R = 0.05
        env = _env(spheres=[np.concatenate([c[s], [R]])])
        cm = orc.state_min_clearance(rb, env, q)
        assert cm <= -(rb.sphere_xyzr[s, 3] + R) + 1e-12
        assert orc.state_collides(rb, env, q) == 1


@pytest.mark.parametrize("L,res,n", [(0.0, 1 / 32, 2), (1 / 32, 1 / 32, 2),
                                     (1 / 32 + 1e-9, 1 / 32, 3), (5.8, 1 / 32, 187),
                                     (0.25, 1 / 32, 9), (1.0, 0.25, 5)])
def test_edge_state_count(orc, L, res, n):
    qa = np.array([0.1, -0.2, 0.3])
    qb = qa + np.array([L * 0.5, -L, 0.0])          # largest per-joint step is L
    assert orc.edge_n_states(qa, qb, res) == n


def test_non_finite_edges_collide(orc):
    """A non-finite joint value makes a state colliding, so an edge with a non-finite endpoint
    collides whatever its other joints do (including an infinite joint span)."""
    w = workload("edges7_shelf", n=4)
    qa, qb = w["qa"].astype(np.float64), w["qb"].astype(np.float64)
    qa[0, 1] = np.nan
    qb[1, 0] = np.inf
    qa[2, 6] = -np.inf
    qb[2, 6] = -np.inf
    flag, cls, emin = orc.edges(w["robot"], w["env"], qa, qb)
    assert list(flag[:3]) == [1, 1, 1] and list(cls[:3]) == [1, 1, 1]
    assert np.isnan(emin[:3]).all()
    assert orc.edge_n_states(qa[1], qb[1], 1 / 32) == 2


def test_edge_states_endpoints_and_spacing(orc):
    g = np.random.default_rng(3)
    for _ in range(20):
        qa, qb = g.uniform(-2.9, 2.9, 7), g.uniform(-2.9, 2.9, 7)
        n = orc.edge_n_states(qa, qb, 1 / 32)
        np.testing.assert_array_equal(orc.edge_state(qa, qb, n, 0), qa)
        np.testing.assert_allclose(orc.edge_state(qa, qb, n, n - 1), qb, atol=1e-15)
        step = np.max(np.abs(orc.edge_state(qa, qb, n, 1) - qa))
        assert step <= 1 / 32 + 1e-15


@pytest.mark.parametrize("name", ["edges7_shelf", "edges8_shelf"])
def test_edge_is_or_of_its_states(orc, name):
    """Second path: materialise each edge's states and validate them as a state batch."""
    w = workload(name, n=48)
    rb, ev = orc.Robot(w["robot"]), orc.Env(w["env"])
    flag, cls, emin = orc.edges(rb, ev, w["qa"], w["qb"], early=False)
    for e in range(len(flag)):
        qa, qb = w["qa"][e].astype(np.float64), w["qb"][e].astype(np.float64)
        n = orc.edge_n_states(qa, qb, 1 / 32)
        qs = np.stack([orc.edge_state(qa, qb, n, k) for k in range(n)], axis=1)
        cm, fl = orc.states(rb, ev, qs)
        assert flag[e] == fl.max()
        assert emin[e] == cm.min()
        assert cls[e] == (1 if cm.min() < -1e-4 else (2 if cm.min() <= 1e-4 else 0))
    # early stop changes the work, not the flag
    flag2, cls2, _ = orc.edges(rb, ev, w["qa"], w["qb"], early=True)
    np.testing.assert_array_equal(flag, flag2)
    np.testing.assert_array_equal(cls, cls2)


def test_explicit_state_count(orc):
    w = workload("edges7_shelf", n=16)
    rb, ev = orc.Robot(w["robot"]), orc.Env(w["env"])
    ns = np.full(16, 2, np.int32)                     # only the two endpoints
    flag, _, emin = orc.edges(rb, ev, w["qa"], w["qb"], n_states=ns, early=False)
    q2 = np.concatenate([w["qa"], w["qb"]]).T.astype(np.float64)
    cm, fl = orc.states(rb, ev, q2)
    np.testing.assert_array_equal(flag, np.maximum(fl[:16], fl[16:]))
    np.testing.assert_array_equal(emin, np.minimum(cm[:16], cm[16:]))


def test_threads_do_not_change_results(orc):
    w = workload("states7", n=256)
    a = orc.states(w["robot"], w["env"], w["q"], n_threads=1)
    b = orc.states(w["robot"], w["env"], w["q"], n_threads=5)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
