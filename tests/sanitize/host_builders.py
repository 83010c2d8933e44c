"""Drive the host-side builders of a host-only sanitizer build of libvk (argv[1]): every robot
and scene the workloads and tests use, through vk_robot_spec_source (the robot program and the
generated specialisation source) and vk_env_describe (primitive records, voxel broadphase,
point grid and clearance field), plus descriptions the builders must reject.  Exits non-zero on
any unexpected result; the sanitizers abort the process on a memory or undefined-behaviour
error."""
import ctypes as C
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import paper_2309_14545_amd as vk  # noqa: E402  (ctypes structures only; libvk.so is not loaded)
from synthetic import workload, rng  # noqa: E402
from synthetic.scenes import cube_scene, random_scene, shelf_scene  # noqa: E402

lib = C.CDLL(sys.argv[1])
lib.vk_robot_spec_source.argtypes = [C.POINTER(vk._RobotDesc), C.c_char_p, C.c_int64]
lib.vk_robot_spec_source.restype = C.c_int64
lib.vk_env_describe.argtypes = [C.POINTER(vk._EnvDesc), C.POINTER(C.c_int64), C.c_int32]
lib.vk_env_describe.restype = C.c_int64
lib.vk_edge_states.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_int32, C.c_float]
lib.vk_edge_states.restype = C.c_int64
lib.vk_last_error.restype = C.c_char_p


def source_len(desc):
    d, _keep = vk._robot_desc(desc)
    n = lib.vk_robot_spec_source(C.byref(d), None, 0)
    if n > 0:
        buf = C.create_string_buffer(int(n))
        assert lib.vk_robot_spec_source(C.byref(d), buf, n) == n
        assert len(buf.value) == n - 1
        small = C.create_string_buffer(17)           # truncated copy, NUL-terminated
        lib.vk_robot_spec_source(C.byref(d), small, 17)
        assert len(small.value) == 16
    return n


def describe(desc):
    d, _keep = vk._env_desc(desc)
    out = (C.c_int64 * 9)()
    return lib.vk_env_describe(C.byref(d), out, 9), list(out)


robots = [workload(n, n=1)["robot"] for n in ("states7", "edges8_shelf", "edges8p_shelf",
                                             "states14_cloud")]
from test_gpu_limits import CASES, _env, _robot  # noqa: E402
robots += [_robot(n, **CASES[n]) for n in CASES]
from test_gpu_long_links import long_robot, scene as long_scene  # noqa: E402
robots.append(long_robot())
for r in robots:
    assert source_len(r) > 1000, lib.vk_last_error()

envs = [{}, workload("states7", n=1)["env"], workload("edges7_shelf", n=1)["env"],
        workload("edges7_shelf_near", n=1)["env"], workload("states14_cloud", n=1)["env"], _env(),
        cube_scene(rng("sanitize", "cube"), n_spheres=3, n_boxes=2),
        shelf_scene(rng("sanitize", "shelf"), n_units=3, n_capsules=5)]
envs += [long_scene(n) for n in ("shelf", "mixed")]
envs += [random_scene(rng("sanitize", f"random{k}")) for k in range(4)]
for e in envs:
    b, stats = describe(e)
    assert b > 0, lib.vk_last_error()

# descriptions the builders reject
base = workload("states7", n=1)["robot"]
bad_robots = [dict(base, dof=0), dict(base, dof=65),
              dict(base, parent_link=np.arange(1, 8, dtype=np.int32)),
              dict(base, sphere_link=np.asarray(base["sphere_link"])[::-1].copy()),
              dict(base, sphere_xyzr=np.where(np.arange(4) == 3, 0.0, np.asarray(base["sphere_xyzr"]))),
              dict(base, dh=np.full_like(np.asarray(base["dh"]), np.nan)),
              dict(base, self_pairs=np.array([[0, 1]], np.int32)),
              dict(base, joint_type=np.full(7, 2, np.int32))]
for r in bad_robots:
    assert source_len(r) == -1, r
box = np.array([[0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1.01, .1, .1, .1]], np.float32)
cyl = np.array([[0, 0, 0, 0, 0, 1.1, .1, .1]], np.float32)
for e in ({"boxes": box}, {"cylinders": cyl}, {"spheres": np.array([[0, 0, 0, -1.0]], np.float32)},
          {"spheres": np.array([[np.nan, 0, 0, .1]], np.float32)}):
    assert describe(e)[0] == -1, e

# the host edge count at its extremes
z = np.zeros(3, np.float32)
fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))  # noqa: E731
far = np.array([0, 0, 3e38], np.float32)
assert lib.vk_edge_states(fp(z), fp(far), 3, C.c_float(1e-30)) == 2 ** 31 - 1
assert lib.vk_edge_states(fp(z), fp(z), 3, C.c_float(1.0 / 32)) == 2
print(f"host builders: {len(robots)} robots, {len(envs)} scenes, "
      f"{len(bad_robots)} + 4 rejected descriptions: ok", flush=True)
