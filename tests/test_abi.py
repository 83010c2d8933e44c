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
    names = re.findall(r"^\s*(?:vk_status|int32_t|const char \*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
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


def test_null_handles_rejected(vk):
    lib = vk.lib()
    assert lib.validate_states(None, None, None, 0, 0, None, None) == -1
    assert lib.validate_edges(None, None, None, None, None, 0, C.c_float(0.03), None, None) == -1
    assert lib.fk_spheres(None, None, 0, 0, None, 0, None) == -1
    assert lib.penetration_cost_fwd(None, None, None, 0, 0, None, None) == -1
    assert lib.vk_robot_destroy(None) == -1
    assert lib.vk_env_destroy(None) == -1
    assert lib.vk_edge_batch_run(None, None) == -1
    assert b"NULL" in lib.vk_last_error()


def test_launch_configuration_checks(vk):
    lib = vk.lib()
    assert lib.vk_set_edge_launch(100, 4) == -1
    assert lib.vk_set_edge_launch(128, 0) == -1
    assert lib.vk_set_edge_launch(1088, 1) == -1
    assert lib.vk_set_edge_launch(1024, 2) == 0
    assert vk.get_edge_launch() == (1024, 2)
    assert lib.vk_set_edge_launch(128, 3) == 0
    assert vk.get_edge_launch() == (128, 3)
    assert lib.vk_set_edge_launch(0, 0) == 0
    assert vk.get_edge_launch() == (256, 4)
    assert lib.vk_set_states_split(1, 1) == -1
    assert lib.vk_set_states_split(-1, 2) == -1
    assert lib.vk_set_states_split(2, 3) == 0
    assert vk.get_states_split() == (2, 3)
    assert lib.vk_set_states_split(0, 1) == 0
