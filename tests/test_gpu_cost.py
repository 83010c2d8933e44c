"""GPU parity of the squared-penetration cost and its adjoint against the FP64 oracle.

Tolerances.  The FP32 sphere centres carry errors of order 1e-6 m; a penetration p shifts by
about that much, so each term p^2 moves by ~2 p * 1e-6, i.e. relatively by 2e-6 / p.  With
penetrations of 1e-2 m and more dominating the sum, the forward check allows an absolute 1e-6
plus a relative 2e-4.  The gradient metric is the per-trajectory relative Frobenius error over
trajectories whose oracle maximum penetration is at least 1e-3 m (there a 1e-6 m centre error
is a small fraction of the penetration); the bound is 1e-4.
"""
import numpy as np
import pytest

from helpers import dev, host, say
from synthetic import workload, rng, chain_robot, bimanual_robot, random_scene, uniform_states

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _cases():
    w = workload("cost7", n=96)                   # 96 trajectories x 64 waypoints
    yield "cost7", w["robot"], w["env"], w["q"], 64
    r14 = workload("states14_cloud", n=1)["robot"]
    env = random_scene(rng("gpu-cost", "env"), mounts=((0, .25, .5), (0, -.25, .5)))
    g = rng("gpu-cost", "cyl")
    cyl = []
    for _ in range(10):
        w_ = g.normal(size=3)
        w_ /= np.linalg.norm(w_)
        cyl.append(np.concatenate([g.uniform(-1, 1, 3), w_, [g.uniform(.05, .3), g.uniform(.03, .15)]]))
    env["cylinders"] = np.asarray(cyl, np.float32)
    yield "bimanual14_mixed", r14, env, uniform_states(rng("gpu-cost", "q14"), 14, 64 * 24), 64
    # prismatic lift + arm, trajectories within each joint's range, shelf scene
    wl = workload("edges8p_shelf", n=1)
    rl = wl["robot"]
    g = rng("gpu-cost", "lift")
    a = g.uniform(rl["q_lo"], rl["q_hi"], (24, 1, 8))
    b = g.uniform(rl["q_lo"], rl["q_hi"], (24, 1, 8))
    t = np.linspace(0.0, 1.0, 64)[None, :, None]
    ql = (a + t * (b - a)).reshape(-1, 8).astype(np.float32)
    yield "lift8_shelf", rl, wl["env"], np.ascontiguousarray(ql.T), 64


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_cost_forward(vk, orc, case):
    name, robot, env, q, _ = case
    say("cost fwd", name, q.shape)
    c = host(vk.penetration_cost_fwd(vk.Robot(robot), vk.Env(env), dev(q))).astype(np.float64)
    ref = orc.costs(robot, env, q)
    err = np.abs(c - ref)
    say("  max abs err", err.max(), "max cost", ref.max(), "active", (ref > 0).mean())
    assert np.all(err <= 1e-6 + 2e-4 * ref)
    cmin, _ = orc.states(robot, env, q)
    assert np.all(c[cmin > 1e-4] == 0.0)         # clearly free states have exactly zero cost


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_cost_gradient(vk, orc, case):
    name, robot, env, q, per = case
    import torch
    n = q.shape[1]
    gc = np.random.default_rng(4).uniform(0.5, 2.0, n).astype(np.float32)
    say("cost bwd", name, q.shape)
    g = host(vk.penetration_cost_bwd(vk.Robot(robot), vk.Env(env), dev(q), dev(gc))).astype(np.float64)
    ref = orc.cost_grads(robot, env, q) * gc[None, :].astype(np.float64)
    cmin, _ = orc.states(robot, env, q)
    # per trajectory (groups of `per` consecutive states)
    checked = 0
    worst = 0.0
    for t in range(n // per):
        sl = slice(t * per, (t + 1) * per)
        if -np.nanmin(cmin[sl]) < 1e-3:
            continue
        rel = np.linalg.norm(g[:, sl] - ref[:, sl]) / np.linalg.norm(ref[:, sl])
        worst = max(worst, rel)
        checked += 1
    glob = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    say(f"  trajectories checked {checked}, worst rel {worst:.2e}, global rel {glob:.2e}")
    assert checked > 0
    assert worst <= 1e-4
    assert glob <= 1e-4
    free = cmin > 1e-4
    assert np.all(g[:, free] == 0.0)


def test_cost_full_size_sampled(vk, orc):
    """The full trajectory batch the benchmark times (4,096 trajectories x 64 waypoints, 262,144
    states) in one launch each way; the oracle checks a seeded sample of 24 trajectories with
    the tolerances above."""
    w = workload("cost7")
    robot, env, q = w["robot"], w["env"], w["q"]
    n, per = q.shape[1], 64
    gc = np.random.default_rng(6).uniform(0.5, 2.0, n).astype(np.float32)
    r, e = vk.Robot(robot), vk.Env(env)
    qd = dev(q)
    c = host(vk.penetration_cost_fwd(r, e, qd)).astype(np.float64)
    g = host(vk.penetration_cost_bwd(r, e, qd, dev(gc))).astype(np.float64)
    say("cost full size", n)
    trajs = np.sort(np.random.default_rng(12).choice(n // per, 24, replace=False))
    cols = (trajs[:, None] * per + np.arange(per)[None, :]).ravel()
    qs = np.ascontiguousarray(q[:, cols])
    ref = orc.costs(robot, env, qs)
    assert np.all(np.abs(c[cols] - ref) <= 1e-6 + 2e-4 * ref)
    gref = orc.cost_grads(robot, env, qs) * gc[cols][None, :].astype(np.float64)
    cmin, _ = orc.states(robot, env, qs)
    checked = 0
    for t in range(len(trajs)):
        sl = slice(t * per, (t + 1) * per)
        if -np.nanmin(cmin[sl]) < 1e-3:
            continue
        gs = g[:, cols[sl]]
        assert np.linalg.norm(gs - gref[:, sl]) <= 1e-4 * np.linalg.norm(gref[:, sl])
        checked += 1
    assert checked > 0
    assert np.all(g[:, cols[cmin > 1e-4]] == 0.0)


def test_autograd_function(vk):
    import torch
    w = workload("cost7", n=8)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    q = dev(w["q"]).requires_grad_(True)
    cost = vk.penetration_cost(q, r, e)
    (2.0 * cost).sum().backward()
    direct = vk.penetration_cost_bwd(r, e, q.detach(), torch.full_like(cost, 2.0))
    torch.testing.assert_close(q.grad, direct, rtol=0, atol=0)


def test_cost_non_finite(vk):
    w = workload("cost7", n=2)
    q = w["q"].copy()
    q[2, 5] = np.nan
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    c = host(vk.penetration_cost_fwd(r, e, dev(q)))
    assert np.isnan(c[5]) and np.isfinite(np.delete(c, 5)).all()
    g = host(vk.penetration_cost_bwd(r, e, dev(q), dev(np.ones(q.shape[1], np.float32))))
    assert np.isnan(g[:, 5]).all() and np.isfinite(np.delete(g, 5, axis=1)).all()


def test_fwd_grad_equals_the_two_calls(vk):
    """penetration_cost_fwd_grad (one adjoint walk) gives bitwise the cost of
    penetration_cost_fwd and the gradient of penetration_cost_bwd with grad_cost = 1; the
    autograd function built on it matches penetration_cost_bwd for any grad_cost."""
    import torch
    w = workload("cost7", n=64)
    q = w["q"].copy()
    q[4, 17] = np.inf
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qd = dev(q)
    n = q.shape[1]
    cost, grad = vk.penetration_cost_fwd_grad(r, e, qd)
    c_ref = host(vk.penetration_cost_fwd(r, e, qd))
    g_ref = host(vk.penetration_cost_bwd(r, e, qd, torch.ones(n, device="cuda")))
    np.testing.assert_array_equal(host(cost), c_ref)
    np.testing.assert_array_equal(host(grad), g_ref)
    assert np.isnan(host(cost)[17]) and (host(cost) > 0).any()
    gc = torch.from_numpy(np.random.default_rng(1).normal(size=n).astype(np.float32)).cuda()
    qg = dev(w["q"]).requires_grad_(True)
    (vk.penetration_cost(qg, r, e) * gc).sum().backward()
    direct = vk.penetration_cost_bwd(r, e, qg.detach(), gc)
    torch.testing.assert_close(qg.grad, direct, rtol=0, atol=0)
    with torch.no_grad():                     # no gradient wanted: the cost kernel alone
        np.testing.assert_array_equal(host(vk.penetration_cost(dev(w["q"]), r, e)),
                                      host(vk.penetration_cost_fwd(r, e, dev(w["q"]))))


def test_adjoint_slots_in_global_memory(vk, orc):
    """A batch that needs more than one round of the adjoint's LDS-bound waves keeps its force
    slots in the stream's workspace (vk_reserve_cost): the cost and gradient equal those of the
    LDS slots (the same sums in the same order), on a stream without the workspace, for the
    262,144-state batch and a ragged size; sampled states agree with the oracle's gradient."""
    import ctypes as C
    import torch
    w = workload("cost7")
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    lib = vk.lib()
    for n in (262144, 200003):
        q = dev(np.ascontiguousarray(w["q"][:, :n]))
        outs = []
        for reserve in (False, True):
            side = torch.cuda.Stream()
            with torch.cuda.stream(side):
                s = C.c_void_p(side.cuda_stream)
                if reserve:
                    assert lib.vk_reserve_cost(s, r.handle, n) == 0
                cost = torch.empty(n, device="cuda")
                grad = torch.empty((7, n), device="cuda")
                assert lib.penetration_cost_fwd_grad(r.handle, e.handle, q.data_ptr(), n, n,
                                                     cost.data_ptr(), grad.data_ptr(), n, s) == 0
                side.synchronize()
                outs.append((host(cost).copy(), host(grad).copy()))
                vk.release(side)
        np.testing.assert_array_equal(outs[0][0], outs[1][0])
        np.testing.assert_array_equal(outs[0][1], outs[1][1])
        say(f"adjoint slots: n {n}, LDS and global slots equal, cost > 0 in "
            f"{(outs[1][0] > 0).mean():.2f} of the states")
    idx = np.arange(0, 262144, 8191)
    ref = orc.cost_grads(w["robot"], w["env"], np.ascontiguousarray(w["q"][:, idx]))
    q = dev(np.ascontiguousarray(w["q"]))
    _, grad = vk.penetration_cost_fwd_grad(r, e, q)           # the binding reserves: global slots
    got = host(grad)[:, idx].astype(np.float64)
    den = max(np.linalg.norm(ref), 1e-30)
    assert np.linalg.norm(got - ref) / den <= 1e-4
