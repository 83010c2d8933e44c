"""GPU parity of fk_spheres and validate_states against the FP64 oracle (through the C ABI)."""
import json
import os

import numpy as np
import pytest

from helpers import BAND, CENTRE_TOL, dev, host, say, state_mismatches
from synthetic import (workload, chain_robot, bimanual_robot, cube_scene, shelf_scene,
                       random_scene, rng, uniform_states)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _robots():
    return {
        "chain7": workload("states7", n=1)["robot"],
        "chain8": workload("edges8_shelf", n=1)["robot"],
        "bimanual14": workload("states14_cloud", n=1)["robot"],
        "lift8": workload("edges8p_shelf", n=1)["robot"],
    }


def _oracle_centres(orc, robot, q):
    rb = orc.Robot(robot)
    return np.stack([orc.sphere_centres(rb, q[:, i]) for i in range(q.shape[1])], axis=2)


def test_fk_hand_values(vk, orc):
    for case in json.load(open(os.path.join(GOLDEN, "fk_hand.json")))["cases"]:
        if "centres" not in case:
            continue
        say("fk hand case", case["name"])
        dh = np.asarray(case["dh"], np.float32)
        sp = np.asarray(case["spheres"], np.float32).reshape(-1, 5)
        robot = {"dof": len(dh), "parent_link": np.asarray(case.get("parent_link", range(len(dh)))),
                 "mount": np.asarray(case["mount"], np.float32) if "mount" in case else None,
                 "dh": dh, "sphere_link": sp[:, 0].astype(np.int32), "sphere_xyzr": sp[:, 1:],
                 "joint_type": np.asarray(case["joint_type"], np.int32) if "joint_type" in case else None}
        r = vk.Robot(robot)
        c = host(vk.fk_spheres(r, dev(np.asarray(case["q"], np.float32).reshape(-1, 1))))
        np.testing.assert_allclose(c[:, :, 0], np.asarray(case["centres"]), atol=CENTRE_TOL)


@pytest.mark.parametrize("name", ["chain7", "chain8", "bimanual14", "lift8"])
def test_fk_spheres_parity(vk, orc, name):
    robot = _robots()[name]
    n = 1037                                  # several 256-lane blocks and a ragged tail
    q = uniform_states(rng("gpu-fk", name), robot["dof"], n)
    if robot.get("joint_type") is not None:   # prismatic strokes within their range
        g = rng("gpu-fk", name + "-range")
        q = np.ascontiguousarray(g.uniform(robot["q_lo"], robot["q_hi"], (n, robot["dof"])).T.astype(np.float32))
    say("fk_spheres", name, "n", n)
    c = host(vk.fk_spheres(vk.Robot(robot), dev(q)))
    ref = _oracle_centres(orc, robot, q.astype(np.float64))
    err = np.linalg.norm(c - ref, axis=1).max()
    say("  max centre error", err)
    assert err <= CENTRE_TOL


def test_fk_spheres_full_size_sampled(vk, orc):
    """2^20 states of the 14-DoF robot in the launch used for large batches; the oracle checks
    a seeded sample of 512 states."""
    robot = _robots()["bimanual14"]
    n = 1 << 20
    q = uniform_states(rng("gpu-fk", "full"), robot["dof"], n)
    say("fk_spheres full size", n)
    c = vk.fk_spheres(vk.Robot(robot), dev(q))
    idx = np.sort(np.random.default_rng(5).choice(n, 512, replace=False))
    sub = host(c[:, :, idx])
    ref = _oracle_centres(orc, robot, q[:, idx].astype(np.float64))
    assert np.linalg.norm(sub - ref, axis=1).max() <= CENTRE_TOL


def test_fk_spheres_leading_dimensions(vk, orc):
    import ctypes as C
    import torch
    robot = _robots()["chain7"]
    r = vk.Robot(robot)
    n, ldq, ldc = 300, 333, 301
    q = np.zeros((robot["dof"], ldq), np.float32)
    q[:, :n] = uniform_states(rng("gpu-fk", "ld"), robot["dof"], n)
    qd = dev(q)
    out = torch.full((r.n_spheres, 3, ldc), -7.0, device="cuda")
    st = vk._stream()
    vk._check(vk.lib().fk_spheres(r.handle, qd.data_ptr(), n, ldq, out.data_ptr(), ldc, st))
    o = host(out)
    ref = _oracle_centres(orc, robot, q[:, :n].astype(np.float64))
    assert np.linalg.norm(o[:, :, :n] - ref, axis=1).max() <= CENTRE_TOL
    assert np.all(o[:, :, n:] == -7.0)       # padding untouched
    assert vk.lib().fk_spheres(r.handle, qd.data_ptr(), n, n - 1, out.data_ptr(), ldc, st) == -2


@pytest.mark.parametrize("theta_off", [0.0, 0.3])
def test_joint_angle_accuracy(vk, theta_off):
    """One revolute joint driving a 1 m link: the sphere at the link's end sits at
    (cos t, sin t, 0) with t = q + theta_off, so its position error is the error of the joint's
    sine and cosine in radians.  Swept densely over several turns and checked against the closed
    form of the FP32 angle the kernel forms, and (within +-7 rad) of the exact angle."""
    desc = dict(dof=1, parent_link=np.array([0], np.int32), mount=None,
                dh=np.array([[1, 0, 1, 0, theta_off]], np.float32),
                sphere_link=np.array([1], np.int32),
                sphere_xyzr=np.array([[0, 0, 0, 0.1]], np.float32),
                self_pairs=np.zeros((0, 2), np.int32))
    r = vk.Robot(desc)
    for hi in (3.2, 7.0, 100.0):
        q = np.linspace(-hi, hi, 1 << 20, dtype=np.float32)
        q[:4] = [0.0, np.float32(np.pi / 2), -np.float32(np.pi), np.float32(1e-30)]
        c = host(vk.fk_spheres(r, dev(q[None, :])))[0]
        t32 = (q + np.float32(theta_off)).astype(np.float64)
        err = np.hypot(c[0] - np.cos(t32), c[1] - np.sin(t32)).max()
        say(f"joint angle error over +-{hi}: {err:.3g} rad")
        assert err <= 1e-6 and np.all(c[2] == 0)
        if hi <= 7.0:
            t = q.astype(np.float64) + np.float64(np.float32(theta_off))
            assert np.hypot(c[0] - np.cos(t), c[1] - np.sin(t)).max() <= 1e-6


def _state_case(name):
    if name == "states7":
        w = workload("states7")
        return w["robot"], w["env"], w["q"]
    if name == "chain8_shelf":
        w = workload("edges8_shelf", n=1)
        return w["robot"], w["env"], uniform_states(rng("gpu-st", name), 8, 2000)
    if name == "bimanual14_cube":
        r = workload("states14_cloud", n=1)["robot"]
        env = cube_scene(rng("gpu-st", "env14"), n_spheres=6, n_boxes=1,
                         mounts=((0, .25, .5), (0, -.25, .5)), sphere_r=(0.02, 0.06))
        return r, env, uniform_states(rng("gpu-st", name), 14, 1037)
    if name == "lift8_shelf":
        w = workload("edges8p_shelf", n=1)
        r = w["robot"]
        g = rng("gpu-st", name)
        q = g.uniform(r["q_lo"], r["q_hi"], (1500, 8)).T.astype(np.float32)
        return r, w["env"], np.ascontiguousarray(q)
    if name == "chain7_mixed_kinds":
        r = workload("states7", n=1)["robot"]
        env = random_scene(rng("gpu-st", "mixed-env"))
        g = rng("gpu-st", "cyl")
        cyl = []
        for _ in range(12):
            w = g.normal(size=3)
            w /= np.linalg.norm(w)
            cyl.append(np.concatenate([g.uniform(-1, 1, 3), w, [g.uniform(.05, .3), g.uniform(.03, .15)]]))
        env["cylinders"] = np.asarray(cyl, np.float32)
        return r, env, uniform_states(rng("gpu-st", name), 7, 1500)
    if name == "chain7_big_env":
        # more records than fit the per-workgroup LDS budget: the global-memory variant runs
        r = workload("states7", n=1)["robot"]
        g = rng("gpu-st", "big")
        c = g.uniform(-4.0, 4.0, (4200, 3))
        env = {"spheres": np.concatenate([c, g.uniform(0.005, 0.02, (4200, 1))], 1).astype(np.float32)}
        return r, env, uniform_states(rng("gpu-st", name), 7, 700)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["states7", "chain8_shelf", "bimanual14_cube",
                                  "chain7_mixed_kinds", "chain7_big_env", "lift8_shelf"])
def test_validate_states_parity(vk, orc, name):
    robot, env, q = _state_case(name)
    say("validate_states", name, "n", q.shape[1])
    flags = host(vk.validate_states(vk.Robot(robot), vk.Env(env), dev(q)))
    cmin, _ = orc.states(robot, env, q)
    bad, near = state_mismatches(flags, cmin)
    say(f"  mismatches outside band {bad}, near-contact {near}, collision rate {flags.mean():.3f}")
    assert bad == 0


@pytest.mark.parametrize("name", ["chain7", "chain8", "bimanual14", "lift8"])
def test_self_only_states_parity(vk, orc, name):
    """No obstacles: every collision is a self-collision, decided through the self-block gates
    alone (both the one-pass and the two-pass schedule)."""
    robot = _robots()[name]
    q = uniform_states(rng("gpu-self", name), robot["dof"], 3001)
    cmin, _ = orc.states(robot, {}, q)
    r, e = vk.Robot(robot), vk.Env({})
    for split in ((0, 1), (1, 2)):
        r.set_states_split(*split)
        flags = host(vk.validate_states(r, e, dev(q)))
        bad, near = state_mismatches(flags, cmin)
        say(f"self-only states {name} split {split}: mismatches {bad}, near {near}, "
            f"rate {flags.mean():.3f}")
        assert bad == 0 and flags.any()


def test_validate_states_non_finite(vk, orc):
    w = workload("states7", n=512)
    q = w["q"].copy()
    q[3, 10] = np.nan
    q[0, 200] = np.inf
    q[6, 511] = -np.inf
    flags = host(vk.validate_states(vk.Robot(w["robot"]), vk.Env(w["env"]), dev(q)))
    assert flags[10] == 1 and flags[200] == 1 and flags[511] == 1
    cmin, _ = orc.states(w["robot"], w["env"], q)
    assert state_mismatches(flags, cmin)[0] == 0


def test_validate_states_empty_and_free(vk):
    import torch
    w = workload("states7", n=64)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    out = vk.validate_states(r, e, torch.zeros((7, 0), device="cuda"))
    assert out.numel() == 0
    # no obstacles and no self pairs: every state is free
    bare = dict(w["robot"])
    bare["self_pairs"] = np.zeros((0, 2), np.int32)
    flags = host(vk.validate_states(vk.Robot(bare), vk.Env({}), dev(w["q"])))
    assert not flags.any()


@pytest.mark.parametrize("name", ["states7", "bimanual14_cube", "chain7_big_env", "lift8_shelf"])
def test_two_pass_schedule_matches_one_pass(vk, name):
    """The two-pass schedule (screen the first link steps, then walk the survivors densely)
    gives bitwise the same flags as one pass, for every split; ragged sizes included."""
    robot, env, q = _state_case(name)
    r, e = vk.Robot(robot), vk.Env(env)
    qd = dev(q)
    ref = host(vk.validate_states(r, e, qd))
    assert r.get_states_split() == (0, 1)
    for num, den in ((1, 3), (1, 2), (2, 3), (9, 10)):
        r.set_states_split(num, den)
        np.testing.assert_array_equal(host(vk.validate_states(r, e, qd)), ref)
        np.testing.assert_array_equal(host(vk.validate_states(r, e, qd[:, :77])), ref[:77])


@pytest.mark.parametrize("name", ["states7", "bimanual14_cube", "chain7_big_env", "lift8_shelf"])
def test_step_ranges_match_the_whole_walk(vk, orc, name):
    """Small batches split over ranges of the walk's tests (each range's waves pose the earlier
    steps and run their own environment parts and self blocks) give bitwise the flags of the
    whole walk, for range counts from two to one per test, at ragged sizes, and the automatic
    choice agrees with the oracle outside the band."""
    robot, env, q = _state_case(name)
    r, e = vk.Robot(robot), vk.Env(env)
    qd = dev(q)
    r.set_states_ranges(0)
    ref = host(vk.validate_states(r, e, qd))
    for k in (2, 3, 5, 16, 23, 32):
        r.set_states_ranges(k)
        for n in (1, 63, 65, q.shape[1]):
            got = host(vk.validate_states(r, e, qd[:, :n].contiguous()))
            np.testing.assert_array_equal(got, ref[:n], err_msg=f"{name} ranges {k} n {n}")
    for bad in (-2, 33):
        with pytest.raises(vk.VkError):
            r.set_states_ranges(bad)
    r.set_states_ranges(-1)
    auto = host(vk.validate_states(r, e, qd))
    np.testing.assert_array_equal(auto, ref)
    cmin, _ = orc.states(robot, env, q)
    bad, near = state_mismatches(auto, cmin)
    say(f"step ranges {name}: {q.shape[1]} states, mismatches {bad}, near {near}")
    assert bad == 0
