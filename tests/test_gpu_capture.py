"""Calls that use the stream's workspace inside HIP graphs: two-pass validate_states and vk_knn
captured on a fresh stream after vk_reserve, replayed several times with eager work and larger
calls (which grow the workspace) between replays, every replay equal to the eager result."""
import ctypes as C

import numpy as np
import pytest

from helpers import dev, host, say
from synthetic import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def test_capture_two_pass_states_and_knn(vk):
    import torch
    w = workload("states7", n=5000)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    r.set_states_split(1, 2)
    q = dev(w["q"])
    g = np.random.default_rng(5)
    x = dev(g.uniform(-2.9, 2.9, (3000, 7)).astype(np.float32))
    ref_f = host(vk.validate_states(r, e, q)).copy()
    ref_i, ref_d = (host(t).copy() for t in vk.knn(x, 10))
    torch.cuda.synchronize()

    side = torch.cuda.Stream()
    vk.reserve(states=5000, knn_samples=3000, knn_k=10, stream=side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="thread_local"):
        # a workspace that would have to grow cannot while the stream is captured
        assert vk.lib().vk_reserve(C.c_void_p(side.cuda_stream), 1 << 26, 0, 0) == -2
        assert b"reserve before the capture" in vk.lib().vk_last_error()
        flags = vk.validate_states(r, e, q)
        idx, d2 = vk.knn(x, 10)
    big_q = dev(workload("states7", n=20000)["q"])
    big_x = dev(g.uniform(-2.9, 2.9, (6000, 7)).astype(np.float32))
    for rep in range(3):
        flags.fill_(7)
        idx.fill_(-7)
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(flags), ref_f)
        np.testing.assert_array_equal(host(idx), ref_i)
        np.testing.assert_array_equal(host(d2), ref_d)
        say("capture replay", rep, "ok")
        # larger calls on the captured stream grow its workspace; the graph keeps its buffer
        with torch.cuda.stream(side):
            vk.validate_states(r, e, big_q[:, : 8000 * (rep + 1)])
            vk.knn(big_x[: 2000 * (rep + 2)], 10)
        torch.cuda.synchronize()
        _ = (q * 2).sum().item()


def test_hot_calls_need_a_workspace(vk):
    """Without vk_reserve on a stream, the calls that need its workspace fail cleanly with
    VK_ERR_SHAPE and enqueue nothing; after it they run."""
    import torch
    w = workload("edges7_shelf", n=64)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    side = torch.cuda.Stream()
    qa, qb = dev(w["qa"]), dev(w["qb"])
    out = torch.empty(64, dtype=torch.uint8, device="cuda")
    s = C.c_void_p(side.cuda_stream)
    st = vk.lib().validate_edges(r.handle, e.handle, qa.data_ptr(), qb.data_ptr(), None, 64,
                                 C.c_float(1.0 / 32.0), out.data_ptr(), s)
    assert st == -2 and b"vk_reserve" in vk.lib().vk_last_error()
    with torch.cuda.stream(side):
        got = host(vk.validate_edges(r, e, qa, qb))      # the binding reserves first
    np.testing.assert_array_equal(got, host(vk.validate_edges(r, e, qa, qb)))
    vk.release(side)
    st = vk.lib().validate_edges(r.handle, e.handle, qa.data_ptr(), qb.data_ptr(), None, 64,
                                 C.c_float(1.0 / 32.0), out.data_ptr(), s)
    assert st == -2


def test_capture_adjoint_with_global_slots(vk):
    """The cost and gradient of a batch large enough to keep the adjoint's force slots in the
    stream's workspace, captured after vk_reserve_cost and replayed with eager work between the
    replays, equal the eager result every time."""
    import torch
    w = workload("cost7")
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    q = dev(np.ascontiguousarray(w["q"]))
    ref_c, ref_g = (host(t).copy() for t in vk.penetration_cost_fwd_grad(r, e, q))
    side = torch.cuda.Stream()
    vk.reserve_cost(r, q.shape[1], stream=side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="thread_local"):
        cost, grad = vk.penetration_cost_fwd_grad(r, e, q)
    for rep in range(3):
        cost.fill_(-1.0)
        grad.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(cost), ref_c)
        np.testing.assert_array_equal(host(grad), ref_g)
        say("adjoint capture replay", rep, "ok")
        _ = (q * 2).sum().item()
