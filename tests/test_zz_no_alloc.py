"""validate_states_noalloc (the allocation-free entry point) against validate_states, through
the C ABI: two calls in a row, the second smaller; a fresh stream with no workspace; a HIP
graph captured without vk_reserve; and the size limit."""
import ctypes as C

import numpy as np
import pytest

from helpers import dev, host, say
from synthetic import workload

pytestmark = pytest.mark.gpu
MAX_STATES = 1 << 22


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _noalloc(vk, r, e, q, n, out, stream):
    return vk.lib().validate_states_noalloc(r.handle, e.handle, q.data_ptr(), n, q.shape[1],
                                            out.data_ptr(), C.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("name,split", [("states7", (1, 2)), ("states7", (0, 1)),
                                        ("states14_cloud", (1, 3))])
def test_noalloc_equals_validate_states(vk, name, split):
    """Two calls in a row on a fresh stream that has no workspace, the second smaller: each
    equals validate_states with the same robot (two-pass with its split, or one pass)."""
    import torch
    w = workload(name, n=40000)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    r.set_states_split(*split)
    q = dev(w["q"])
    side = torch.cuda.Stream()
    for n in (40000, 3001):
        ref = host(vk.validate_states(r, e, q[:, :n].contiguous()))
        out = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        qn = q[:, :n].contiguous()
        torch.cuda.synchronize()
        assert _noalloc(vk, r, e, qn, n, out, side) == 0, vk.lib().vk_last_error()
        side.synchronize()
        got = host(out)
        say(f"noalloc {name} split {split} n {n}: rate {got.mean():.3f}")
        np.testing.assert_array_equal(got, ref)


def test_noalloc_in_a_graph_without_reserve(vk):
    """Captured on a fresh stream that never had vk_reserve, replayed three times with eager
    work and another no-alloc call of a different size between replays."""
    import torch
    w = workload("states7", n=9000)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    r.set_states_split(1, 3)
    q = dev(w["q"])
    ref = host(vk.validate_states(r, e, q))
    other = q[:, :1234].contiguous()
    ref_other = host(vk.validate_states(r, e, other))
    out = torch.full((9000,), 7, dtype=torch.uint8, device="cuda")
    out_other = torch.empty(1234, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="thread_local"):
        assert _noalloc(vk, r, e, q, 9000, out, side) == 0
    for rep in range(3):
        out.fill_(7)
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(out), ref)
        assert _noalloc(vk, r, e, other, 1234, out_other, torch.cuda.current_stream()) == 0
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(out_other), ref_other)
        _ = (q * 2).sum().item()


def test_noalloc_size_limit(vk):
    """More states than the fixed scratch holds: VK_ERR_SHAPE before anything is enqueued."""
    import torch
    w = workload("states7", n=64)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    q = dev(w["q"])
    out = torch.empty(64, dtype=torch.uint8, device="cuda")
    st = vk.lib().validate_states_noalloc(r.handle, e.handle, q.data_ptr(), MAX_STATES + 1,
                                          MAX_STATES + 1, out.data_ptr(), None)
    assert st == -2 and b"maximum" in vk.lib().vk_last_error()
    assert vk.lib().validate_states_noalloc(r.handle, e.handle, q.data_ptr(), 0, 0,
                                            out.data_ptr(), None) == 0
