"""GPU parity for robots whose links are longer than the environment's voxel lists cover.

The voxel broadphase lists, per cell, the primitives within 0.5 m; a link step whose bounding
sphere is larger than that tests every primitive behind its bounding sphere instead (the
mid-phase of Sec. III-D applied to the whole primitive list), in the collision walk and in
the cost walks.  This file drives those branches: a chain of 1.2 m links, eight spheres each, in
the shelf scene and in a scene of spheres, capsules, cylinders and boxes.  Centres, state
flags, edge flags, cost and gradient are held to the bars of the other parity tests.
"""
import numpy as np
import pytest

from helpers import BAND, CENTRE_TOL, dev, host, say, state_mismatches
from synthetic import rng, workload
from synthetic.scenes import random_scene

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0
VOXEL_REACH = 0.5        # the distance up to which the voxel lists hold primitives (metres)


def long_robot():
    """4-DoF chain of 1.2 m links (twists 0, +90, -90, 0 degrees), 8 spheres along each link,
    self pairs between links at least two apart."""
    g = rng("gpu-long", "robot")
    dof, per, a = 4, 8, 1.2
    tw = [0.0, np.pi / 2, -np.pi / 2, 0.0]
    dh = np.array([[a, 0.05, np.cos(t), np.sin(t), 0.0] for t in tw])
    link, xyzr = [], []
    for l in range(1, dof + 1):
        for k in range(per):
            u = (k + 0.5) / per
            xyzr.append([-a * u, g.uniform(-0.02, 0.02), g.uniform(-0.02, 0.02),
                         g.uniform(0.04, 0.08)])
            link.append(l)
    link = np.asarray(link, np.int32)
    pairs = [(i, j) for i in range(len(link)) for j in range(i + 1, len(link))
             if abs(int(link[i]) - int(link[j])) >= 2]
    return {"dof": dof, "parent_link": np.arange(dof, dtype=np.int32),
            "mount": np.tile(np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32), (dof, 1)),
            "dh": dh.astype(np.float32),
            "q_lo": np.full(dof, -np.pi, np.float32), "q_hi": np.full(dof, np.pi, np.float32),
            "sphere_link": link, "sphere_xyzr": np.asarray(xyzr, np.float32),
            "self_pairs": np.asarray(pairs, np.int32).reshape(-1, 2)}


def link_bound_radii(robot):
    """Bounding radius of each link's spheres as the library forms it: the centre of their
    axis-aligned box, the radius reaching the farthest sphere surface."""
    out = []
    for l in np.unique(robot["sphere_link"]):
        s = robot["sphere_xyzr"][robot["sphere_link"] == l].astype(np.float64)
        c = 0.5 * ((s[:, :3] - s[:, 3:]).min(0) + (s[:, :3] + s[:, 3:]).max(0))
        out.append(float((np.linalg.norm(s[:, :3] - c, axis=1) + s[:, 3]).max()))
    return np.asarray(out)


def scene(name):
    if name == "shelf":
        return workload("edges7_shelf", n=1)["env"]
    env = random_scene(rng("gpu-long", "mixed"), lo=60, hi=60)
    g = rng("gpu-long", "cylinders")
    cyl = []
    for _ in range(10):
        w = g.normal(size=3)
        w /= np.linalg.norm(w)
        cyl.append(np.concatenate([g.uniform(-1.5, 1.5, 3), w, [g.uniform(0.05, 0.3), g.uniform(0.03, 0.15)]]))
    env["cylinders"] = np.asarray(cyl, np.float32)
    return env


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def test_links_exceed_the_voxel_reach():
    radii = link_bound_radii(long_robot())
    assert np.all(radii > VOXEL_REACH), radii


def test_long_link_centres(vk, orc):
    robot = long_robot()
    q = rng("gpu-long", "centres").uniform(-np.pi, np.pi, (robot["dof"], 300)).astype(np.float32)
    got = host(vk.fk_spheres(vk.Robot(robot), dev(q)))
    want = np.stack([orc.sphere_centres(robot, q[:, i]) for i in range(q.shape[1])], axis=2)
    err = np.sqrt(((got.astype(np.float64) - want) ** 2).sum(axis=1)).max()
    say(f"long links: centre error {err:.2e} m")
    assert err <= CENTRE_TOL


@pytest.mark.parametrize("name", ["shelf", "mixed"])
def test_long_link_states(vk, orc, name):
    robot, env = long_robot(), scene(name)
    q = rng("gpu-long", "states-" + name).uniform(-np.pi, np.pi, (robot["dof"], 2000)).astype(np.float32)
    flags = host(vk.validate_states(vk.Robot(robot), vk.Env(env), dev(q)))
    cmin, _ = orc.states(robot, env, q)
    bad, near = state_mismatches(flags, cmin)
    say(f"long links {name}: collision rate {flags.mean():.3f}, mismatches {bad}, near {near}")
    assert bad == 0 and 0.05 < flags.mean() < 0.95


@pytest.mark.parametrize("name", ["shelf", "mixed"])
def test_long_link_edges(vk, orc, name):
    robot, env = long_robot(), scene(name)
    g = rng("gpu-long", "edges-" + name)
    qa = g.uniform(-np.pi, np.pi, (300, robot["dof"])).astype(np.float32)
    qb = (qa + g.uniform(-0.6, 0.6, qa.shape)).astype(np.float32)
    flags = host(vk.validate_edges(vk.Robot(robot), vk.Env(env), dev(qa), dev(qb), resolution=RES))
    _, _, emin = orc.edges(robot, env, qa, qb, res=RES, early=False)
    bad, near = state_mismatches(flags, emin)
    say(f"long links {name} edges: collision rate {flags.mean():.3f}, mismatches {bad}, near {near}")
    assert bad == 0 and 0.05 < flags.mean() < 0.95


@pytest.mark.parametrize("name", ["shelf", "mixed"])
def test_long_link_cost(vk, orc, name):
    """Cost (1e-6 + 2e-4 relative) and gradient (1e-4 relative per trajectory that penetrates
    by at least 1 mm, and overall; exact zeros where the state is clearly free)."""
    robot, env = long_robot(), scene(name)
    g = rng("gpu-long", "traj-" + name)
    n_traj, per, dof = 16, 32, robot["dof"]
    a = g.uniform(-np.pi, np.pi, (n_traj, 1, dof))
    b = a + g.uniform(-0.5, 0.5, (n_traj, 1, dof))
    t = np.linspace(0.0, 1.0, per)[None, :, None]
    q = np.ascontiguousarray((a + t * (b - a)).reshape(-1, dof).T.astype(np.float32))
    r, e = vk.Robot(robot), vk.Env(env)
    c = host(vk.penetration_cost_fwd(r, e, dev(q))).astype(np.float64)
    ref = orc.costs(robot, env, q)
    assert np.all(np.abs(c - ref) <= 1e-6 + 2e-4 * ref)
    gc = np.random.default_rng(9).uniform(0.5, 2.0, q.shape[1]).astype(np.float32)
    grad = host(vk.penetration_cost_bwd(r, e, dev(q), dev(gc))).astype(np.float64)
    gref = orc.cost_grads(robot, env, q) * gc[None, :].astype(np.float64)
    cmin, _ = orc.states(robot, env, q)
    worst, checked = 0.0, 0
    for k in range(n_traj):
        sl = slice(k * per, (k + 1) * per)
        if -np.nanmin(cmin[sl]) < 1e-3:
            continue
        worst = max(worst, np.linalg.norm(grad[:, sl] - gref[:, sl]) / np.linalg.norm(gref[:, sl]))
        checked += 1
    glob = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
    say(f"long links {name} cost: active {(ref > 0).mean():.3f}, trajectories checked {checked}, "
        f"worst rel {worst:.2e}, global rel {glob:.2e}")
    assert checked > 0 and worst <= 1e-4 and glob <= 1e-4
    free = cmin > BAND
    assert np.all(c[free] == 0.0) and np.all(grad[:, free] == 0.0)
