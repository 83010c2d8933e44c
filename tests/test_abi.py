"""C-ABI checks that need no GPU: the library loads, exports every function include/vk.h
declares, and rejects bad descriptions and handles before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vk.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:vk_status|int32_t|int64_t|const char \*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def vk():
    import paper_2309_14545_amd as vk
    if not os.path.exists(vk.LIB_PATH):
        from paper_2309_14545_amd import build
        build.build()
    return vk


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fk_spheres", "validate_states", "validate_edges", "penetration_cost_fwd",
                 "penetration_cost_bwd", "vk_robot_create", "vk_env_create", "vk_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(vk):
    lib = vk.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(vk.EXPORTS)


def _robot_desc(vk, **over):
    dof = 2
    base = dict(dof=dof, parent_link=np.array([0, 1], np.int32), mount=None,
                dh=np.array([[1, 0, 1, 0, 0], [1, 0, 1, 0, 0]], np.float32),
                sphere_link=np.array([1, 2], np.int32),
                sphere_xyzr=np.array([[0, 0, 0, 0.1], [0, 0, 0, 0.1]], np.float32),
                self_pairs=np.zeros((0, 2), np.int32))
    base.update(over)
    return base


@pytest.mark.parametrize("bad", [
    dict(dof=0),
    dict(parent_link=np.array([0, 2], np.int32)),
    dict(sphere_link=np.array([2, 1], np.int32)),
    dict(sphere_link=np.array([1, 3], np.int32)),
    dict(sphere_xyzr=np.array([[0, 0, 0, 0.1], [0, 0, 0, 0.0]], np.float32)),
    dict(sphere_xyzr=np.array([[0, 0, 0, 0.1], [np.nan, 0, 0, 0.1]], np.float32)),
    dict(self_pairs=np.array([[0, 5]], np.int32)),
    dict(sphere_link=np.array([1, 1], np.int32), self_pairs=np.array([[0, 1]], np.int32)),
    dict(dh=np.array([[1, 0, 1, 0, 0], [np.inf, 0, 1, 0, 0]], np.float32)),
])
def test_bad_robot_descriptions_are_rejected(vk, bad):
    with pytest.raises(vk.VkError) as e:
        vk.Robot(_robot_desc(vk, **bad))
    assert e.value.status == -1
    assert vk.lib().vk_last_error()


def test_too_many_joints_unsupported(vk):
    dof = 65
    d = dict(dof=dof, parent_link=np.arange(dof, dtype=np.int32), mount=None,
             dh=np.tile(np.array([1, 0, 1, 0, 0], np.float32), (dof, 1)),
             sphere_link=np.zeros(0, np.int32), sphere_xyzr=np.zeros((0, 4), np.float32))
    with pytest.raises(vk.VkError) as e:
        vk.Robot(d)
    assert e.value.status == -3


def test_bad_environment_rejected(vk):
    with pytest.raises(vk.VkError):
        vk.Env({"spheres": np.array([[0, 0, 0, -1.0]], np.float32)})
    with pytest.raises(vk.VkError):
        vk.Env({"boxes": np.full((1, 15), np.nan, np.float32)})


def test_primitive_frames_must_be_unit(vk):
    """A cylinder axis off unit length, or a box rotation off orthonormal, by more than 1e-5 is
    rejected before anything reaches the device; FP32 roundings of exact ones are accepted."""
    axis = np.array([0.0, 0.6, 0.8]) * (1.0 + 3e-5)
    cyl = np.array([[0, 0, 0, *axis, 0.1, 0.1]], np.float32)
    with pytest.raises(vk.VkError) as e:
        vk.Env({"cylinders": cyl})
    assert e.value.status == -1 and b"axis" in vk.lib().vk_last_error()
    R = np.array([[1, 0, 0], [0, 1, 2e-4], [0, 0, 1]])
    box = np.array([[0, 0, 0, *R.reshape(-1), 0.1, 0.1, 0.1]], np.float32)
    with pytest.raises(vk.VkError) as e:
        vk.Env({"boxes": box})
    assert e.value.status == -1 and b"orthonormal" in vk.lib().vk_last_error()
    c, s = np.cos(0.3), np.sin(0.3)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]) * (1.0 + 2e-7)
    # a mirror (det -1) is orthonormal too: the distance does not depend on handedness
    ok_box = np.array([[0, 0, 0, *R.reshape(-1), 0.1, 0.1, 0.1]], np.float32)
    try:
        vk.Env({"boxes": ok_box, "cylinders": np.array([[0, 0, 0, 0, 0.6, 0.8, 0.1, 0.1]], np.float32)})
    except vk.VkError as err:
        # without a device the checks pass and the upload fails with a HIP error
        assert err.status in (-4, -5), err


def test_edge_state_count_on_the_host(vk, orc):
    """vk_edge_states: the hand cases of the edge discretisation (Sec. III-D), saturation for
    endpoints very far apart, invalid input, and agreement with the oracle's count."""
    z = np.zeros(3, np.float32)
    res = 1.0 / 32.0
    assert vk.edge_states(z, z, res) == 2
    assert vk.edge_states(z, np.array([0, res, 0], np.float32), res) == 2
    assert vk.edge_states(z, np.array([0, np.nextafter(np.float32(res), np.float32(1)), 0], np.float32), res) == 3
    assert vk.edge_states(z, np.array([0, 2.9, 0], np.float32), res) == 94
    assert vk.edge_states(np.array([-2.9], np.float32), np.array([2.9], np.float32), res) == 187
    assert vk.edge_states(z, np.array([0, 0, 1e9], np.float32), res) == 2 ** 31 - 1
    assert vk.edge_states(z, np.array([0, 0, np.nan], np.float32), res) == -1
    assert vk.edge_states(z, z, 0.0) == -1
    assert vk.edge_states(z, z, float("inf")) == -1
    g = np.random.default_rng(8)
    qa = g.uniform(-2.9, 2.9, (500, 7)).astype(np.float32)
    qb = g.uniform(-2.9, 2.9, (500, 7)).astype(np.float32)
    for r in (1.0 / 32.0, 1.0 / 256.0, 0.1):
        mine = [vk.edge_states(qa[e], qb[e], r) for e in range(len(qa))]
        assert mine == orc.edge_n_states_batch(qa, qb, r).tolist()


def test_null_handles_rejected(vk):
    lib = vk.lib()
    assert lib.validate_states(None, None, None, 0, 0, None, None) == -1
    assert lib.validate_edges(None, None, None, None, None, 0, C.c_float(0.03), None, None) == -1
    assert lib.fk_spheres(None, None, 0, 0, None, 0, None) == -1
    assert lib.penetration_cost_fwd(None, None, None, 0, 0, None, None) == -1
    assert lib.vk_robot_destroy(None) == -1
    assert lib.vk_env_destroy(None) == -1
    assert lib.vk_edge_batch_run(None, None, None, None, None) == -1
    assert lib.vk_robot_set_edge_launch(None, 256, 4, 8) == -1
    assert lib.vk_autotune_edges(None, None, None, None, None, 0, C.c_float(0.03), None, 0, None) == -1
    assert b"NULL" in lib.vk_last_error()


def test_launch_configuration_checks(vk):
    """Launch settings are checked before the handle: invalid values are named as such."""
    lib = vk.lib()
    for args in ((100, 4, 8), (128, 0, 8), (1088, 1, 8), (256, 4, 0), (256, 4, 65), (64, 65, 8)):
        assert lib.vk_robot_set_edge_launch(None, *args) == -1
        assert b"robot handle" not in lib.vk_last_error(), args
    for args in ((1024, 2, 8), (128, 3, 1), (0, 0, 0)):
        assert lib.vk_robot_set_edge_launch(None, *args) == -1
        assert b"robot handle" in lib.vk_last_error(), args
    for num, den in ((1, 1), (-1, 2), (0, 0)):
        assert lib.vk_robot_set_states_split(None, num, den) == -1
        assert b"num < den" in lib.vk_last_error()
    assert lib.vk_robot_set_states_split(None, 2, 3) == -1
    assert b"robot handle" in lib.vk_last_error()


def test_reserve_argument_checks(vk):
    lib = vk.lib()
    assert lib.vk_reserve(None, -1, 0, 0) == -1
    assert lib.vk_reserve(None, 0, -5, 0) == -1
    assert lib.vk_reserve(None, 0, 100, 33) == -1
    assert lib.vk_reserve(None, 1 << 31, 0, 0) == -2
    assert lib.vk_reserve_cost(None, None, 10) == -1          # NULL robot
    assert b"robot" in lib.vk_last_error()


def test_specialisation_source_is_exact(vk):
    """vk_robot_spec_source needs no device: the 7-DoF robot's generated source names its step
    count and carries every sphere as exact hexadecimal floats."""
    import re
    from synthetic import workload
    robot = workload("states7", n=1)["robot"]
    src = vk.spec_source(robot)
    steps = int(re.search(r"static constexpr int n_steps = (\d+);", src).group(1))
    assert steps >= robot["dof"]            # at least one step per moving link
    body = src[src.index("spheres["):src.index("};", src.index("spheres["))]
    rows = re.findall(r"float4\{([^}]*)\}", body)
    xyzr = np.asarray(robot["sphere_xyzr"], np.float32)
    assert len(rows) == len(xyzr) + 8       # eight records of padding for the register slots
    got = np.array([[float.fromhex(v.strip().rstrip("f")) for v in r.split(",")] for r in rows],
                   np.float32)
    np.testing.assert_array_equal(got[:len(xyzr)], xyzr)
    assert not got[len(xyzr):].any()
    assert "vk_spec_edges_counted_2" in src
    bad = dict(robot, sphere_link=np.asarray(robot["sphere_link"])[::-1].copy())
    with pytest.raises(vk.VkError):
        vk.spec_source(bad)
