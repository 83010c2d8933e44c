"""Python binding of libvk (the C ABI in include/vk.h): argument marshalling only.

Every step of the validation path runs in the HIP kernels of libvk.so; PyTorch supplies device
memory and the current stream.  Importing this module does not need a GPU, but every call
that enqueues work needs the built library and a HIP device, and fails loudly otherwise.

Layouts follow the C ABI: a batch of configurations is SoA ``[dof, N]`` float32; edge endpoints
are ``[E, dof]`` float32; flags are uint8 (1 = in collision).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvk.so")

VK_OK = 0
_STATUS = {-1: "VK_ERR_INVALID_ARG", -2: "VK_ERR_SHAPE", -3: "VK_ERR_UNSUPPORTED",
           -4: "VK_ERR_HIP", -5: "VK_ERR_OOM"}

EXPORTS = ("vk_robot_create", "vk_robot_destroy", "vk_robot_dof", "vk_robot_n_spheres",
           "vk_robot_specialize", "vk_robot_use_specialized", "vk_robot_is_specialized",
           "vk_robot_spec_source",
           "vk_env_create", "vk_env_destroy", "vk_env_describe", "vk_edge_states", "fk_spheres", "validate_states",
           "validate_states_noalloc", "validate_edges",
           "validate_edges_per_edge", "validate_edges_counted", "validate_edges_indexed",
           "vk_knn", "vk_knn_pairs", "vk_tree_nearest", "vk_tree_steer", "vk_tree_append",
           "vk_rrt_extend", "vk_rrt_commit", "vk_shortcut_propose", "vk_shortcut_apply",
           "penetration_cost_fwd", "penetration_cost_bwd", "penetration_cost_fwd_grad",
           "vk_edge_batch_create", "vk_edge_batch_run", "vk_edge_batch_get_launch",
           "vk_edge_batch_destroy", "vk_reserve", "vk_reserve_cost", "vk_release",
           "vk_robot_set_edge_launch", "vk_robot_get_edge_launch", "vk_robot_set_edge_parts",
           "vk_robot_get_edge_parts", "vk_robot_set_states_split",
           "vk_robot_get_states_split", "vk_robot_set_states_ranges", "vk_robot_get_states_ranges",
           "vk_robot_set_edge_ranges", "vk_robot_get_edge_ranges",
           "vk_autotune_edges", "vk_autotune_states",
           "vk_last_error")


class VkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _RobotDesc(C.Structure):
    _fields_ = [("dof", C.c_int32), ("parent_link", C.POINTER(C.c_int32)),
                ("mount", C.POINTER(C.c_float)), ("dh", C.POINTER(C.c_float)),
                ("q_lo", C.POINTER(C.c_float)), ("q_hi", C.POINTER(C.c_float)),
                ("n_spheres", C.c_int32), ("sphere_link", C.POINTER(C.c_int32)),
                ("sphere_xyzr", C.POINTER(C.c_float)), ("n_self_pairs", C.c_int32),
                ("self_pairs", C.POINTER(C.c_int32)), ("joint_type", C.POINTER(C.c_int32))]


class _EnvDesc(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("spheres", C.POINTER(C.c_float)),
                ("n_capsules", C.c_int32), ("capsules", C.POINTER(C.c_float)),
                ("n_cylinders", C.c_int32), ("cylinders", C.POINTER(C.c_float)),
                ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_float))]


class _EdgeSet(C.Structure):
    _fields_ = [("robot", C.c_int32), ("env", C.c_int32), ("qa_offset", C.c_int64),
                ("n_edges", C.c_int64), ("out_offset", C.c_int64)]


_lib = None


def lib():
    """Load libvk.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2309_14545_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, fp = C.c_void_p, C.c_int64, C.c_int32, C.c_float
        L.vk_robot_create.argtypes = [C.POINTER(_RobotDesc), C.POINTER(vp)]
        L.vk_robot_destroy.argtypes = [vp]
        L.vk_robot_dof.argtypes = [vp]
        L.vk_robot_dof.restype = i32
        L.vk_robot_n_spheres.argtypes = [vp]
        L.vk_robot_n_spheres.restype = i32
        L.vk_robot_specialize.argtypes = [vp, C.c_char_p]
        L.vk_robot_use_specialized.argtypes = [vp, i32]
        L.vk_robot_is_specialized.argtypes = [vp]
        L.vk_robot_is_specialized.restype = i32
        L.vk_robot_spec_source.argtypes = [C.POINTER(_RobotDesc), C.c_char_p, i64]
        L.vk_robot_spec_source.restype = i64
        L.vk_env_create.argtypes = [C.POINTER(_EnvDesc), C.POINTER(vp)]
        L.vk_env_destroy.argtypes = [vp]
        L.vk_env_describe.argtypes = [C.POINTER(_EnvDesc), C.POINTER(i64), i32]
        L.vk_env_describe.restype = i64
        L.vk_edge_states.argtypes = [C.POINTER(fp), C.POINTER(fp), i32, fp]
        L.vk_edge_states.restype = i64
        L.fk_spheres.argtypes = [vp, vp, i64, i64, vp, i64, vp]
        L.validate_states.argtypes = [vp, vp, vp, i64, i64, vp, vp]
        L.validate_states_noalloc.argtypes = [vp, vp, vp, i64, i64, vp, vp]
        L.validate_edges.argtypes = [vp, vp, vp, vp, vp, i64, fp, vp, vp]
        L.validate_edges_per_edge.argtypes = [vp, vp, vp, vp, vp, i64, fp, vp, vp]
        L.validate_edges_counted.argtypes = [vp, vp, vp, vp, vp, i64, fp, vp, vp, vp]
        L.validate_edges_indexed.argtypes = [vp, vp, vp, i64, vp, vp, i64, fp, vp, vp]
        L.vk_knn.argtypes = [vp, i64, i32, i32, vp, vp, vp]
        L.vk_knn_pairs.argtypes = [vp, i64, i32, vp, vp]
        L.vk_tree_nearest.argtypes = [vp, vp, i32, i32, i64, vp, vp, vp, vp]
        L.vk_tree_steer.argtypes = [vp, i32, i32, i64, vp, vp, fp, vp, vp, vp]
        L.vk_tree_append.argtypes = [vp, vp, vp, i32, i32, i64, vp, vp, vp, vp, vp]
        L.vk_rrt_extend.argtypes = [vp, vp, i32, i32, i64, vp, vp, fp, vp, vp, vp, vp, vp]
        L.vk_rrt_commit.argtypes = [vp, vp, vp, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                    vp, vp, vp]
        L.vk_shortcut_propose.argtypes = [vp, i64, i32, i32, vp, vp, vp]
        L.vk_shortcut_apply.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, vp, vp]
        L.penetration_cost_fwd.argtypes = [vp, vp, vp, i64, i64, vp, vp]
        L.penetration_cost_bwd.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp]
        L.penetration_cost_fwd_grad.argtypes = [vp, vp, vp, i64, i64, vp, vp, i64, vp]
        L.vk_edge_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp), i32,
                                           C.POINTER(_EdgeSet), i32, fp, i32, i32, C.POINTER(vp)]
        L.vk_edge_batch_run.argtypes = [vp, vp, vp, vp, vp]
        L.vk_edge_batch_get_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.vk_edge_batch_destroy.argtypes = [vp]
        L.vk_reserve.argtypes = [vp, i64, i64, i32]
        L.vk_reserve_cost.argtypes = [vp, vp, i64]
        L.vk_release.argtypes = [vp]
        L.vk_robot_set_edge_launch.argtypes = [vp, i32, i32, i32]
        L.vk_robot_get_edge_launch.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.vk_robot_set_edge_parts.argtypes = [vp, i32]
        L.vk_robot_get_edge_parts.argtypes = [vp]
        L.vk_robot_get_edge_parts.restype = i32
        L.vk_robot_set_states_split.argtypes = [vp, i32, i32]
        L.vk_robot_get_states_split.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.vk_robot_set_states_ranges.argtypes = [vp, i32]
        L.vk_robot_set_edge_ranges.argtypes = [vp, i32]
        L.vk_robot_get_edge_ranges.argtypes = [vp]
        L.vk_robot_get_edge_ranges.restype = i32
        L.vk_robot_get_states_ranges.argtypes = [vp, C.POINTER(i32)]
        L.vk_autotune_edges.argtypes = [vp, vp, vp, vp, vp, i64, fp, C.c_char_p, i32, vp]
        L.vk_autotune_states.argtypes = [vp, vp, vp, i64, i64, C.c_char_p, i32, vp]
        L.vk_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("vk_robot_dof", "vk_robot_n_spheres", "vk_last_error", "vk_edge_states",
                            "vk_robot_is_specialized", "vk_robot_spec_source", "vk_env_describe",
                            "vk_robot_get_edge_parts"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(status: int):
    if status != VK_OK:
        raise VkError(status, lib().vk_last_error().decode())


def _f32(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(shape))


def _i32(a, shape):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(shape))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


def _robot_desc(desc: dict):
    """(vk_robot_desc, the arrays it points into) for a dict of numpy arrays."""
    dof = int(desc["dof"])
    keep = {
        "parent_link": _i32(desc["parent_link"], (-1,)) if desc.get("parent_link") is not None else None,
        "mount": _f32(desc["mount"], (-1, 12)) if desc.get("mount") is not None else None,
        "dh": _f32(desc["dh"], (-1, 5)),
        "sphere_link": _i32(desc["sphere_link"], (-1,)),
        "sphere_xyzr": _f32(desc["sphere_xyzr"], (-1, 4)),
        "self_pairs": _i32(desc.get("self_pairs", np.zeros((0, 2))), (-1, 2)),
        "joint_type": _i32(desc["joint_type"], (-1,)) if desc.get("joint_type") is not None else None,
    }
    d = _RobotDesc(dof, _ip(keep["parent_link"]), _fp(keep["mount"]), _fp(keep["dh"]), None,
                   None, len(keep["sphere_link"]), _ip(keep["sphere_link"]),
                   _fp(keep["sphere_xyzr"]), len(keep["self_pairs"]), _ip(keep["self_pairs"]),
                   _ip(keep["joint_type"]))
    return d, keep


def spec_source(desc: dict) -> str:
    """The source vk_robot_specialize compiles for this robot description (no device needed)."""
    d, _keep = _robot_desc(desc)
    n = lib().vk_robot_spec_source(C.byref(d), None, 0)
    if n < 0:
        raise VkError(-1, lib().vk_last_error().decode())
    buf = C.create_string_buffer(int(n))
    lib().vk_robot_spec_source(C.byref(d), buf, n)
    return buf.value.decode()


class Robot:
    """Device-resident robot (see vk_robot_desc).  ``desc`` is a dict of numpy arrays."""

    def __init__(self, desc: dict):
        dof = int(desc["dof"])
        d, keep = _robot_desc(desc)
        h = C.c_void_p()
        _check(lib().vk_robot_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.dof = dof
        self.n_spheres = len(keep["sphere_link"])

    def specialize(self, cache_dir: str | None = None):
        """Compile this robot's edge kernels with its program as constants (vk_robot_specialize)
        and use them; cache_dir keeps the code objects between processes."""
        _check(lib().vk_robot_specialize(self.handle, cache_dir.encode() if cache_dir else None))

    def use_specialized(self, on: bool = True):
        _check(lib().vk_robot_use_specialized(self.handle, 1 if on else 0))

    @property
    def specialized(self) -> bool:
        return lib().vk_robot_is_specialized(self.handle) == 1

    def set_edge_launch(self, block_threads: int = 0, blocks_per_cu: int = 0,
                        tickets_per_wave: int = 0):
        """Launch shape of this robot's edge launches (all 0: the defaults 256, 4, 8)."""
        _check(lib().vk_robot_set_edge_launch(self.handle, int(block_threads), int(blocks_per_cu),
                                              int(tickets_per_wave)))

    def set_edge_parts(self, parts: int = 1):
        """Waves sharing one edge's rake (long edges); 1 = one wave per edge."""
        _check(lib().vk_robot_set_edge_parts(self.handle, int(parts)))

    @property
    def edge_parts(self) -> int:
        return int(lib().vk_robot_get_edge_parts(self.handle))

    def set_edge_ranges(self, max_ranges: int = -1):
        """Test ranges of small edge batches (-1 automatic, 0 or 1 never, k at most k <= 32)."""
        _check(lib().vk_robot_set_edge_ranges(self.handle, int(max_ranges)))

    def edge_ranges(self) -> int:
        return int(lib().vk_robot_get_edge_ranges(self.handle))

    def get_edge_launch(self):
        b, p, t = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().vk_robot_get_edge_launch(self.handle, C.byref(b), C.byref(p), C.byref(t)))
        return b.value, p.value, t.value

    def set_states_split(self, num: int, den: int = 1):
        """Two-pass schedule of validate_states for this robot; (0, 1) = one pass."""
        _check(lib().vk_robot_set_states_split(self.handle, int(num), int(den)))

    def set_states_ranges(self, max_ranges: int = -1):
        """Test ranges of small state batches (-1 automatic, 0 or 1 never, k at most k <= 32)."""
        _check(lib().vk_robot_set_states_ranges(self.handle, int(max_ranges)))

    def get_states_split(self):
        n, d = C.c_int32(), C.c_int32()
        _check(lib().vk_robot_get_states_split(self.handle, C.byref(n), C.byref(d)))
        return n.value, d.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vk_robot_destroy(self.handle)
            self.handle = None


def _env_desc(desc: dict):
    """(vk_env_desc, the arrays it points into) for a dict of numpy arrays."""
    arrs = {}
    for key, w in (("spheres", 4), ("capsules", 7), ("cylinders", 8), ("boxes", 15)):
        a = desc.get(key)
        arrs[key] = _f32(a if a is not None else np.zeros((0, w)), (-1, w))
    d = _EnvDesc(len(arrs["spheres"]), _fp(arrs["spheres"]), len(arrs["capsules"]),
                 _fp(arrs["capsules"]), len(arrs["cylinders"]), _fp(arrs["cylinders"]),
                 len(arrs["boxes"]), _fp(arrs["boxes"]))
    return d, arrs


ENV_FIELDS = ("spheres", "capsules", "cylinders", "boxes", "points", "voxel_cells",
              "voxel_entries", "grid_cells", "field_cells")


def env_describe(desc: dict) -> dict:
    """vk_env_describe: what vk_env_create would build (no device needed)."""
    d, _keep = _env_desc(desc)
    out = (C.c_int64 * len(ENV_FIELDS))()
    b = lib().vk_env_describe(C.byref(d), out, len(ENV_FIELDS))
    if b < 0:
        raise VkError(-1, lib().vk_last_error().decode())
    return dict(zip(ENV_FIELDS, list(out)), device_bytes=int(b))


class Env:
    """Device-resident environment (see vk_env_desc)."""

    def __init__(self, desc: dict):
        d, arrs = _env_desc(desc)
        h = C.c_void_p()
        _check(lib().vk_env_create(C.byref(d), C.byref(h)))
        self.handle = h
        self.counts = {k: len(v) for k, v in arrs.items()}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vk_env_destroy(self.handle)
            self.handle = None


def edge_states(qa, qb, resolution: float = 1.0 / 32.0) -> int:
    """States validate_edges gives the edge qa -> qb (host arrays [dof]); -1 for invalid input."""
    a, b = _f32(qa, (-1,)), _f32(qb, (-1,))
    if a.shape != b.shape:
        raise ValueError("qa and qb must have the same length")
    return int(lib().vk_edge_states(_fp(a), _fp(b), len(a), float(resolution)))


# --- device tensors ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


# Workspace sizes reserved so far per (device, stream): (states, knn samples, knn k).
_reserved = {}


def reserve(states: int = 0, knn_samples: int = 0, knn_k: int = 0, stream=None):
    """vk_reserve for the current (or given) torch stream: the workspace of calls of up to
    these sizes.  A set-up call: do it before capturing a graph on the stream."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    key = (torch.cuda.current_device(), st.cuda_stream)
    have = _reserved.get(key, (0, 0, 0))
    want = (max(have[0], int(states)), max(have[1], int(knn_samples)), max(have[2], int(knn_k)))
    if key in _reserved and want == have:
        return
    _check(lib().vk_reserve(C.c_void_p(st.cuda_stream), *want))
    _reserved[key] = want


_reserved_cost = {}


def reserve_cost(robot, states: int, stream=None):
    """vk_reserve_cost for the current (or given) torch stream: the adjoint's workspace for up to
    `states` states of `robot` (large batches keep its force slots there instead of in LDS).  A
    set-up call: do it before capturing a graph on the stream."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    per = _reserved_cost.setdefault((torch.cuda.current_device(), st.cuda_stream), {})
    key = robot.handle.value                  # the handle's address
    if per.get(key, -1) >= int(states):
        return
    _check(lib().vk_reserve_cost(C.c_void_p(st.cuda_stream), robot.handle, int(states)))
    per[key] = int(states)


def release(stream=None):
    """vk_release for the current (or given) torch stream."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    _reserved.pop((torch.cuda.current_device(), st.cuda_stream), None)
    _reserved_cost.pop((torch.cuda.current_device(), st.cuda_stream), None)
    _check(lib().vk_release(C.c_void_p(st.cuda_stream)))


def _dev_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 CUDA (HIP) tensor")
    return t.contiguous()


def _soa(robot, q, name="q"):
    q = _dev_f32(q, name)
    if q.dim() != 2 or q.shape[0] != robot.dof:
        raise ValueError(f"{name} must be [dof={robot.dof}, N] (structure of arrays)")
    return q


def fk_spheres(robot: Robot, q):
    """Sphere centres [S, 3, N] of the SoA batch q [dof, N]."""
    torch = _torch()
    q = _soa(robot, q)
    n = q.shape[1]
    out = torch.empty((robot.n_spheres, 3, n), dtype=torch.float32, device=q.device)
    _check(lib().fk_spheres(robot.handle, q.data_ptr(), n, n, out.data_ptr(), n, _stream()))
    return out


def validate_states(robot: Robot, env: Env, q):
    """Collision flags uint8 [N] of the SoA batch q [dof, N]."""
    torch = _torch()
    q = _soa(robot, q)
    n = q.shape[1]
    out = torch.empty(n, dtype=torch.uint8, device=q.device)
    if robot.get_states_split()[0] > 0:
        reserve(states=n)
    _check(lib().validate_states(robot.handle, env.handle, q.data_ptr(), n, n, out.data_ptr(),
                                 _stream()))
    return out


def validate_states_noalloc(robot: Robot, env: Env, q, out):
    """validate_states into the caller's uint8 [N] tensor ``out``, allocating nothing (the
    two-pass schedule with the library's fixed scratch array; N <= 2^22)."""
    q = _soa(robot, q)
    n = q.shape[1]
    _check(lib().validate_states_noalloc(robot.handle, env.handle, q.data_ptr(), n, n,
                                         out.data_ptr(), _stream()))
    return out


def validate_edges(robot: Robot, env: Env, qa, qb, n_states=None, resolution: float = 1.0 / 32.0,
                   per_edge: bool = False, out=None):
    """Edge collision flags uint8 [E] for endpoints qa, qb [E, dof].

    ``per_edge=True`` uses one kernel launch per edge (the baseline); otherwise all edges run
    in one persistent launch."""
    torch = _torch()
    qa, qb = _dev_f32(qa, "qa"), _dev_f32(qb, "qb")
    if qa.dim() != 2 or qa.shape != qb.shape or qa.shape[1] != robot.dof:
        raise ValueError(f"qa and qb must both be [E, dof={robot.dof}]")
    E = qa.shape[0]
    ns_ptr = None
    if n_states is not None:
        if not (isinstance(n_states, torch.Tensor) and n_states.is_cuda and n_states.dtype == torch.int32
                and n_states.shape == (E,)):
            raise TypeError("n_states must be an int32 CUDA tensor [E]")
        n_states = n_states.contiguous()
        ns_ptr = n_states.data_ptr()
    if out is None:
        out = torch.empty(E, dtype=torch.uint8, device=qa.device)
    fn = lib().validate_edges_per_edge if per_edge else lib().validate_edges
    if not per_edge:
        reserve()
    _check(fn(robot.handle, env.handle, qa.data_ptr(), qb.data_ptr(), ns_ptr, E, float(resolution),
              out.data_ptr(), _stream()))
    return out


def validate_edges_counted(robot: Robot, env: Env, qa, qb, flops, n_states=None,
                           resolution: float = 1.0 / 32.0, out=None):
    """validate_edges plus executed-FLOP accounting into ``flops`` (int64 CUDA tensor [8]:
    total, FK, culling, fine environment tests, self pairs, re-posing, surplus rake lanes, rake
    slots of real states walked)."""
    torch = _torch()
    qa, qb = _dev_f32(qa, "qa"), _dev_f32(qb, "qb")
    if qa.dim() != 2 or qa.shape != qb.shape or qa.shape[1] != robot.dof:
        raise ValueError(f"qa and qb must both be [E, dof={robot.dof}]")
    if not (isinstance(flops, torch.Tensor) and flops.is_cuda and flops.dtype == torch.int64
            and flops.numel() >= 8 and flops.is_contiguous()):
        raise TypeError("flops must be a contiguous int64 CUDA tensor of 8 elements")
    E = qa.shape[0]
    ns_ptr = n_states.contiguous().data_ptr() if n_states is not None else None
    if out is None:
        out = torch.empty(E, dtype=torch.uint8, device=qa.device)
    reserve()
    _check(lib().validate_edges_counted(robot.handle, env.handle, qa.data_ptr(), qb.data_ptr(),
                                        ns_ptr, E, float(resolution), out.data_ptr(),
                                        flops.data_ptr(), _stream()))
    return out


def validate_edges_indexed(robot: Robot, env: Env, nodes, pairs, n_states=None,
                           resolution: float = 1.0 / 32.0, out=None):
    """Edge flags uint8 [E] for edges between rows of ``nodes`` [N, dof] given by ``pairs``
    (int32 [E, 2]; a pair with a negative entry is a hole, flag 0)."""
    torch = _torch()
    nodes = _dev_f32(nodes, "nodes")
    if nodes.dim() != 2 or nodes.shape[1] != robot.dof:
        raise ValueError(f"nodes must be [N, dof={robot.dof}]")
    if not (isinstance(pairs, torch.Tensor) and pairs.is_cuda and pairs.dtype == torch.int32
            and pairs.dim() == 2 and pairs.shape[1] == 2):
        raise TypeError("pairs must be an int32 CUDA tensor [E, 2]")
    pairs = pairs.contiguous()
    E = pairs.shape[0]
    ns_ptr = None
    if n_states is not None:
        if not (isinstance(n_states, torch.Tensor) and n_states.is_cuda and n_states.dtype == torch.int32
                and n_states.shape == (E,)):
            raise TypeError("n_states must be an int32 CUDA tensor [E]")
        n_states = n_states.contiguous()
        ns_ptr = n_states.data_ptr()
    if out is None:
        out = torch.empty(E, dtype=torch.uint8, device=nodes.device)
    reserve()
    _check(lib().validate_edges_indexed(robot.handle, env.handle, nodes.data_ptr(), nodes.shape[0],
                                        pairs.data_ptr(), ns_ptr, E, float(resolution),
                                        out.data_ptr(), _stream()))
    return out


def knn(x, k: int):
    """(idx int32 [N, k], dist2 float32 [N, k]): the k nearest other rows of x [N, dim]."""
    torch = _torch()
    x = _dev_f32(x, "x")
    if x.dim() != 2:
        raise ValueError("x must be [N, dim]")
    n, d = x.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=x.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=x.device)
    if 1 <= k <= 32:
        reserve(knn_samples=n, knn_k=k)
    _check(lib().vk_knn(x.data_ptr(), n, d, k, idx.data_ptr(), d2.data_ptr(), _stream()))
    return idx, d2


def knn_pairs(idx):
    """Undirected roadmap edges int32 [N*k, 2] from kNN lists (holes are (-1, -1))."""
    torch = _torch()
    if not (isinstance(idx, torch.Tensor) and idx.is_cuda and idx.dtype == torch.int32 and idx.dim() == 2):
        raise TypeError("idx must be an int32 CUDA tensor [N, k]")
    idx = idx.contiguous()
    n, k = idx.shape
    pairs = torch.empty((n * k, 2), dtype=torch.int32, device=idx.device)
    _check(lib().vk_knn_pairs(idx.data_ptr(), n, k, pairs.data_ptr(), _stream()))
    return pairs


def tree_nearest(nodes, sizes, targets, active=None, out=None):
    """Index [Q] of the node of each query's tree (nodes [Q, cap, dof], sizes [Q]) nearest to
    targets [Q, dof]; -1 for empty trees or inactive queries."""
    torch = _torch()
    Q, cap, dof = nodes.shape
    if out is None:
        out = torch.empty(Q, dtype=torch.int32, device=nodes.device)
    _check(lib().vk_tree_nearest(nodes.data_ptr(), sizes.data_ptr(), cap, dof, Q,
                                 targets.data_ptr(), active.data_ptr() if active is not None else None,
                                 out.data_ptr(), _stream()))
    return out


def tree_steer(nodes, near, targets, step: float, qnew=None, reached=None):
    """(qnew [Q, dof], reached uint8 [Q]): a step of at most `step` from node near[q] toward
    targets[q]."""
    torch = _torch()
    Q, cap, dof = nodes.shape
    if qnew is None:
        qnew = torch.empty((Q, dof), dtype=torch.float32, device=nodes.device)
    if reached is None:
        reached = torch.empty(Q, dtype=torch.uint8, device=nodes.device)
    _check(lib().vk_tree_steer(nodes.data_ptr(), cap, dof, Q, near.data_ptr(), targets.data_ptr(),
                               float(step), qnew.data_ptr(), reached.data_ptr(), _stream()))
    return qnew, reached


def tree_append(nodes, parents, sizes, qnew, near, ok, added=None):
    """Append qnew[q] (parent near[q]) to the trees where ok[q]; returns the new indices (-1 where
    nothing was added)."""
    torch = _torch()
    Q, cap, dof = nodes.shape
    if added is None:
        added = torch.empty(Q, dtype=torch.int32, device=nodes.device)
    _check(lib().vk_tree_append(nodes.data_ptr(), parents.data_ptr(), sizes.data_ptr(), cap, dof, Q,
                                qnew.data_ptr(), near.data_ptr(), ok.data_ptr(), added.data_ptr(),
                                _stream()))
    return added


def rrt_extend(nodes, sizes, targets, active, step: float, qnear, qnew, near, reached):
    """One fused extension of every active query's tree (nodes [Q, cap, dof], sizes [Q]) toward
    targets [Q, dof]: fills near [Q], reached [Q] and the edge qnear -> qnew ([Q, dof] each) that
    validate_edges checks next.  Inactive queries get a zero-length edge and near = -1."""
    Q, cap, dof = nodes.shape
    _check(lib().vk_rrt_extend(nodes.data_ptr(), sizes.data_ptr(), cap, dof, Q, targets.data_ptr(),
                               active.data_ptr(), float(step), qnear.data_ptr(), qnew.data_ptr(),
                               near.data_ptr(), reached.data_ptr(), _stream()))


def rrt_commit(nodes, parents, sizes, qnew, near, reached, flags, going, added, edges,
               from_added=None, meet_this=None, meet_from=None, solved=None):
    """Bookkeeping after an extension's edges were checked (flags [Q]): appends the free ones'
    new nodes (added [Q], -1 where none), counts the going queries' edges into edges (int64 [1])
    and updates going [Q] in place.  With from_added (the other tree's nodes added this
    iteration) a node added at its target joins the trees: solved, meet_this and meet_from are
    set for those queries."""
    Q, cap, dof = nodes.shape
    ptr = lambda t: t.data_ptr() if t is not None else None   # noqa: E731
    _check(lib().vk_rrt_commit(nodes.data_ptr(), parents.data_ptr(), sizes.data_ptr(), cap, dof, Q,
                               qnew.data_ptr(), near.data_ptr(), reached.data_ptr(),
                               flags.data_ptr(), going.data_ptr(), added.data_ptr(),
                               ptr(from_added), ptr(meet_this), ptr(meet_from), ptr(solved),
                               edges.data_ptr(), _stream()))


def shortcut_propose(lens, max_len: int, k: int, rnd, pairs=None):
    """k shortcut candidates per path as node index pairs [P * k, 2] (see vk_shortcut_propose);
    rnd: int32/uint32 CUDA tensor of 2 * P * k random words."""
    torch = _torch()
    P = lens.shape[0]
    if pairs is None:
        pairs = torch.empty((P * k, 2), dtype=torch.int32, device=lens.device)
    _check(lib().vk_shortcut_propose(lens.data_ptr(), P, int(max_len), int(k), rnd.data_ptr(),
                                     pairs.data_ptr(), _stream()))
    return pairs


def shortcut_apply(paths, lens, k: int, pairs, flags, accepted=None):
    """Splice each path's best valid candidate into paths [P, M, dof] / lens [P] in place."""
    P, M, dof = paths.shape
    _check(lib().vk_shortcut_apply(paths.data_ptr(), lens.data_ptr(), P, M, dof, int(k),
                                   pairs.data_ptr(), flags.data_ptr(),
                                   accepted.data_ptr() if accepted is not None else None,
                                   _stream()))
    return accepted


def penetration_cost_fwd(robot: Robot, env: Env, q):
    """Squared-penetration cost float32 [N] of the SoA batch q [dof, N]."""
    torch = _torch()
    q = _soa(robot, q)
    n = q.shape[1]
    out = torch.empty(n, dtype=torch.float32, device=q.device)
    _check(lib().penetration_cost_fwd(robot.handle, env.handle, q.data_ptr(), n, n,
                                      out.data_ptr(), _stream()))
    return out


def penetration_cost_bwd(robot: Robot, env: Env, q, grad_cost):
    """grad_q [dof, N] = grad_cost[i] * d cost_i / d q."""
    torch = _torch()
    q = _soa(robot, q)
    n = q.shape[1]
    g = _dev_f32(grad_cost, "grad_cost")
    if g.shape != (n,):
        raise ValueError("grad_cost must be [N]")
    out = torch.empty((robot.dof, n), dtype=torch.float32, device=q.device)
    reserve_cost(robot, n)
    _check(lib().penetration_cost_bwd(robot.handle, env.handle, q.data_ptr(), n, n, g.data_ptr(),
                                      out.data_ptr(), n, _stream()))
    return out


def penetration_cost_fwd_grad(robot: Robot, env: Env, q):
    """(cost [N], d cost / d q [dof, N]) from one adjoint launch."""
    torch = _torch()
    q = _soa(robot, q)
    n = q.shape[1]
    cost = torch.empty(n, dtype=torch.float32, device=q.device)
    grad = torch.empty((robot.dof, n), dtype=torch.float32, device=q.device)
    reserve_cost(robot, n)
    _check(lib().penetration_cost_fwd_grad(robot.handle, env.handle, q.data_ptr(), n, n,
                                           cost.data_ptr(), grad.data_ptr(), n, _stream()))
    return cost, grad


def _make_cost_function():
    torch = _torch()

    class PenetrationCost(torch.autograd.Function):
        """cost = PenetrationCost.apply(q, robot, env): differentiable in q ([dof, N]).  When q
        needs a gradient, the forward runs the adjoint walk once (cost and d cost / d q), and
        the backward scales that gradient by grad_cost; otherwise the forward runs the cost
        kernel alone."""

        @staticmethod
        def forward(ctx, q, robot, env):
            if not ctx.needs_input_grad[0]:
                return penetration_cost_fwd(robot, env, q)
            cost, grad = penetration_cost_fwd_grad(robot, env, q)
            ctx.save_for_backward(grad)
            return cost

        @staticmethod
        def backward(ctx, grad_cost):
            (grad,) = ctx.saved_tensors
            return grad * grad_cost.reshape(1, -1), None, None

    return PenetrationCost


_PC = None


def penetration_cost(q, robot: Robot, env: Env):
    """Autograd entry point: cost [N] whose backward runs the adjoint kernel."""
    global _PC
    if _PC is None:
        _PC = _make_cost_function()
    return _PC.apply(q, robot, env)


class EdgeBatch:
    """Mixed-robot edge batch replayed from a HIP graph (vk_edge_batch_*); the launch shape is
    fixed at creation (block, per_cu both 0: the defaults)."""

    def __init__(self, robots, envs, sets, resolution: float = 1.0 / 32.0, block: int = 0,
                 per_cu: int = 0):
        self._keep = (list(robots), list(envs))
        rh = (C.c_void_p * len(robots))(*[r.handle.value for r in robots])
        eh = (C.c_void_p * len(envs))(*[e.handle.value for e in envs])
        st = (_EdgeSet * len(sets))(*[_EdgeSet(*s) for s in sets])
        h = C.c_void_p()
        _check(lib().vk_edge_batch_create(rh, len(robots), eh, len(envs), st, len(sets),
                                          float(resolution), int(block), int(per_cu), C.byref(h)))
        self.handle = h

    def run(self, qa, qb, out):
        """Replay on device arrays qa, qb (float32) and out (uint8) holding every set's edges."""
        self._arrays = (qa, qb, out)          # kept alive until the next run
        _check(lib().vk_edge_batch_run(self.handle, qa.data_ptr(), qb.data_ptr(), out.data_ptr(),
                                       _stream()))

    def launch(self):
        b, p = C.c_int32(), C.c_int32()
        _check(lib().vk_edge_batch_get_launch(self.handle, C.byref(b), C.byref(p)))
        return b.value, p.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.vk_edge_batch_destroy(self.handle)
            self.handle = None
