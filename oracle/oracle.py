"""ctypes binding of the FP64 reference oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg; never by the library.  Inputs are the canonical FP32 arrays of the synthetic
workloads, upcast to float64 here so the oracle and the GPU path start from identical values.

Every function returns numpy arrays; see ``oracle.c`` for the definitions and the passages of
the paper they follow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD_PATH = os.path.join(_HERE, "liboracle.so")
# The planted-mistake tests point this at a mutated build of oracle.c; nothing else sets it.
_LIB_PATH = os.environ.get("VK_ORACLE_LIB") or _BUILD_PATH
_lib = None

SPHERE, CAPSULE, CYLINDER, BOX = 0, 1, 2, 3
BAND = 1e-4


CFLAGS = ["-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared", "-pthread"]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2: no fast-math, no vector intrinsics)."""
    if force or not os.path.exists(_BUILD_PATH):
        tmp = _BUILD_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _BUILD_PATH)
    return _BUILD_PATH


class _Robot(C.Structure):
    _fields_ = [("dof", C.c_int), ("parent_link", C.POINTER(C.c_int32)),
                ("mount", C.POINTER(C.c_double)), ("dh", C.POINTER(C.c_double)),
                ("n_spheres", C.c_int), ("sphere_link", C.POINTER(C.c_int32)),
                ("sphere_xyzr", C.POINTER(C.c_double)), ("n_pairs", C.c_int),
                ("pairs", C.POINTER(C.c_int32)), ("joint_type", C.POINTER(C.c_int32))]


class _Env(C.Structure):
    _fields_ = [("n_spheres", C.c_int), ("spheres", C.POINTER(C.c_double)),
                ("n_capsules", C.c_int), ("capsules", C.POINTER(C.c_double)),
                ("n_cylinders", C.c_int), ("cylinders", C.POINTER(C.c_double)),
                ("n_boxes", C.c_int), ("boxes", C.POINTER(C.c_double))]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lib_handle():
    global _lib
    if _lib is None:
        if _LIB_PATH == _BUILD_PATH and (not os.path.exists(_LIB_PATH) or
                                         os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        lib = C.CDLL(_LIB_PATH)
        R, E = C.POINTER(_Robot), C.POINTER(_Env)
        dp, i64, u8p = C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_uint8)
        lib.orc_fk.argtypes = [R, dp, dp, dp]
        lib.orc_sphere_centres.argtypes = [R, dp, dp]
        for name in ("orc_sd_sphere", "orc_sd_capsule", "orc_sd_cylinder", "orc_sd_box"):
            getattr(lib, name).argtypes = [dp, dp]
            getattr(lib, name).restype = C.c_double
        lib.orc_clearance.argtypes = [C.c_int, dp, C.c_double, dp]
        lib.orc_clearance.restype = C.c_double
        lib.orc_state_min_clearance.argtypes = [R, E, dp]
        lib.orc_state_min_clearance.restype = C.c_double
        lib.orc_state_collides.argtypes = [R, E, dp]
        lib.orc_state_collides.restype = C.c_int
        lib.orc_edge_n_states.argtypes = [dp, dp, C.c_int, C.c_double]
        lib.orc_edge_n_states.restype = C.c_int
        lib.orc_edge_state.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, dp]
        lib.orc_cost.argtypes = [R, E, dp]
        lib.orc_cost.restype = C.c_double
        lib.orc_cost_grad.argtypes = [R, E, dp, dp]
        lib.orc_states.argtypes = [R, E, dp, i64, i64, dp, u8p, C.c_int]
        lib.orc_edges.argtypes = [R, E, dp, dp, C.POINTER(C.c_int32), i64, C.c_double, u8p,
                                  C.POINTER(C.c_int8), dp, C.c_int, C.c_int]
        lib.orc_costs.argtypes = [R, E, dp, i64, i64, dp, C.c_int]
        lib.orc_cost_grads.argtypes = [R, E, dp, i64, i64, dp, i64, C.c_int]
        lib.orc_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape) if shape is not None else a


class Robot:
    """Oracle-side copy of a robot description (FP64)."""

    def __init__(self, desc: dict):
        dof = int(desc["dof"])
        self.dof = dof
        self.parent_link = np.ascontiguousarray(desc["parent_link"], dtype=np.int32)
        mount = desc.get("mount")
        if mount is None:
            mount = np.tile(np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0.0]), (dof, 1))
        self.mount = _f64(mount, (dof, 12))
        self.dh = _f64(desc["dh"], (dof, 5))
        self.sphere_link = np.ascontiguousarray(desc["sphere_link"], dtype=np.int32)
        self.sphere_xyzr = _f64(desc["sphere_xyzr"], (-1, 4))
        self.pairs = np.ascontiguousarray(np.asarray(desc["self_pairs"], dtype=np.int32).reshape(-1, 2))
        self.n_spheres = len(self.sphere_link)
        jt = desc.get("joint_type")
        self.joint_type = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
        self.c = _Robot(dof, _ip(self.parent_link), _dp(self.mount), _dp(self.dh),
                        self.n_spheres, _ip(self.sphere_link), _dp(self.sphere_xyzr),
                        len(self.pairs), _ip(self.pairs),
                        None if self.joint_type is None else _ip(self.joint_type))


class Env:
    """Oracle-side copy of an environment (FP64)."""

    def __init__(self, desc: dict):
        self.spheres = _f64(desc.get("spheres", np.zeros((0, 4))), (-1, 4))
        self.capsules = _f64(desc.get("capsules", np.zeros((0, 7))), (-1, 7))
        self.cylinders = _f64(desc.get("cylinders", np.zeros((0, 8))), (-1, 8))
        self.boxes = _f64(desc.get("boxes", np.zeros((0, 15))), (-1, 15))
        self.c = _Env(len(self.spheres), _dp(self.spheres), len(self.capsules),
                      _dp(self.capsules), len(self.cylinders), _dp(self.cylinders),
                      len(self.boxes), _dp(self.boxes))


def _as_robot(r):
    return r if isinstance(r, Robot) else Robot(r)


def _as_env(e):
    return e if isinstance(e, Env) else Env(e)


def threads(n: int = 0) -> int:
    return _lib_handle().orc_threads(n)


def fk(robot, q):
    """Link transforms [(dof+1), 3, 4] and joint frames [dof, 3, 4] for one configuration."""
    rb = _as_robot(robot)
    q = _f64(q, (rb.dof,))
    T = np.zeros((rb.dof + 1, 12))
    P = np.zeros((rb.dof, 12))
    _lib_handle().orc_fk(C.byref(rb.c), _dp(q), _dp(T), _dp(P))
    return T.reshape(-1, 3, 4), P.reshape(-1, 3, 4)


def sphere_centres(robot, q):
    rb = _as_robot(robot)
    q = _f64(q, (rb.dof,))
    out = np.zeros((rb.n_spheres, 3))
    _lib_handle().orc_sphere_centres(C.byref(rb.c), _dp(q), _dp(out))
    return out


def sd(kind: int, point, prim) -> float:
    p, pr = _f64(point, (3,)), _f64(prim)
    f = ("orc_sd_sphere", "orc_sd_capsule", "orc_sd_cylinder", "orc_sd_box")[kind]
    return getattr(_lib_handle(), f)(_dp(p), _dp(pr))


def clearance(kind: int, centre, radius: float, prim) -> float:
    p, pr = _f64(centre, (3,)), _f64(prim)
    return _lib_handle().orc_clearance(kind, _dp(p), float(radius), _dp(pr))


def state_min_clearance(robot, env, q) -> float:
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q, (rb.dof,))
    return _lib_handle().orc_state_min_clearance(C.byref(rb.c), C.byref(ev.c), _dp(q))


def state_collides(robot, env, q) -> int:
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q, (rb.dof,))
    return _lib_handle().orc_state_collides(C.byref(rb.c), C.byref(ev.c), _dp(q))


def states(robot, env, q_soa, n_threads: int = 0):
    """Minimum clearance and flag per state; q_soa is [dof][N]."""
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q_soa)
    n = q.shape[1]
    cmin = np.zeros(n)
    flag = np.zeros(n, dtype=np.uint8)
    _lib_handle().orc_states(C.byref(rb.c), C.byref(ev.c), _dp(q), n, n, _dp(cmin),
                             flag.ctypes.data_as(C.POINTER(C.c_uint8)), n_threads)
    return cmin, flag


def edge_n_states(qa, qb, res: float) -> int:
    a, b = _f64(qa), _f64(qb)
    return _lib_handle().orc_edge_n_states(_dp(a), _dp(b), len(a), float(res))


def edge_n_states_batch(qa, qb, res: float) -> np.ndarray:
    qa, qb = _f64(qa), _f64(qb)
    return np.array([edge_n_states(qa[e], qb[e], res) for e in range(len(qa))], dtype=np.int32)


def edge_state(qa, qb, n: int, k: int):
    a, b = _f64(qa), _f64(qb)
    out = np.zeros(len(a))
    _lib_handle().orc_edge_state(_dp(a), _dp(b), len(a), int(n), int(k), _dp(out))
    return out


def edges(robot, env, qa, qb, res: float = 1.0 / 32.0, n_states=None, early: bool = True,
          n_threads: int = 0):
    """Edge flag (OR over states), class (0 free, 1 colliding, 2 near contact) and minimum
    clearance; qa/qb are AoS [E][dof]."""
    rb, ev = _as_robot(robot), _as_env(env)
    a, b = _f64(qa, (-1, rb.dof)), _f64(qb, (-1, rb.dof))
    E = a.shape[0]
    flag = np.zeros(E, dtype=np.uint8)
    cls = np.zeros(E, dtype=np.int8)
    emin = np.zeros(E)
    ns = None
    ns_p = None
    if n_states is not None:
        ns = np.ascontiguousarray(n_states, dtype=np.int32)
        ns_p = _ip(ns)
    _lib_handle().orc_edges(C.byref(rb.c), C.byref(ev.c), _dp(a), _dp(b), ns_p, E, float(res),
                            flag.ctypes.data_as(C.POINTER(C.c_uint8)),
                            cls.ctypes.data_as(C.POINTER(C.c_int8)), _dp(emin),
                            1 if early else 0, n_threads)
    return flag, cls, emin


def cost(robot, env, q) -> float:
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q, (rb.dof,))
    return _lib_handle().orc_cost(C.byref(rb.c), C.byref(ev.c), _dp(q))


def cost_grad(robot, env, q):
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q, (rb.dof,))
    g = np.zeros(rb.dof)
    _lib_handle().orc_cost_grad(C.byref(rb.c), C.byref(ev.c), _dp(q), _dp(g))
    return g


def costs(robot, env, q_soa, n_threads: int = 0):
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q_soa)
    n = q.shape[1]
    out = np.zeros(n)
    _lib_handle().orc_costs(C.byref(rb.c), C.byref(ev.c), _dp(q), n, n, _dp(out), n_threads)
    return out


def cost_grads(robot, env, q_soa, n_threads: int = 0):
    """Analytic FP64 gradient [dof][N]."""
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q_soa)
    n = q.shape[1]
    g = np.zeros((rb.dof, n))
    _lib_handle().orc_cost_grads(C.byref(rb.c), C.byref(ev.c), _dp(q), n, n, _dp(g), n,
                                 n_threads)
    return g


def cost_grad_fd(robot, env, q, h: float = 1e-6):
    """Central finite differences of the FP64 cost."""
    rb, ev = _as_robot(robot), _as_env(env)
    q = _f64(q, (rb.dof,))
    g = np.zeros(rb.dof)
    for j in range(rb.dof):
        qp, qm = q.copy(), q.copy()
        qp[j] += h
        qm[j] -= h
        g[j] = (cost(rb, ev, qp) - cost(rb, ev, qm)) / (2.0 * h)
    return g
