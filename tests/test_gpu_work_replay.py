"""The instrumented edge kernel's rake-slot count against a CPU replay of the rake schedule
(Sec. III-D, Fig. 2): lane l takes state l * ceil(n / 64) + k at step k (a lane past the end
repeats the last state, so a step with such a lane also checks state n - 1), and the edge ends
after the first step in which some lane's state collides.  The replay takes every state's collision
from the FP64 oracle, so it shares nothing with the kernel; edges with a state in the
near-contact band are left out (their exit step is not fixed by the oracle)."""
import numpy as np
import pytest

from helpers import BAND, dev, host, say
from synthetic import workload

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0
W = 64


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _states_of(qa, qb, counts):
    """Every state q_k = qa + k / (n - 1) (qb - qa) of every edge, FP64, SoA [dof][sum n]."""
    a = qa.astype(np.float64)
    b = qb.astype(np.float64)
    e = np.repeat(np.arange(len(qa)), counts)
    k = np.concatenate([np.arange(n) for n in counts])
    t = k / (np.repeat(counts, counts) - 1.0)
    q = a[e] + t[:, None] * (b[e] - a[e])
    return np.ascontiguousarray(q.T), e, k


def _replay(counts, collide):
    """Rake slots of real states walked per edge, and the edge flags, from per-state flags."""
    visits = np.zeros(len(counts), np.int64)
    flags = np.zeros(len(counts), np.uint8)
    start = 0
    for i, n in enumerate(counts):
        c = collide[start:start + n]
        start += n
        stride = -(-n // W)
        for k in range(stride):
            idx = np.arange(W) * stride + k
            surplus = (idx >= n).any()
            idx = idx[idx < n]
            visits[i] += len(idx)
            if c[idx].any() or (surplus and c[n - 1]):
                flags[i] = 1
                break
    return visits, flags


def test_rake_slots_match_the_replay(vk, orc):
    import torch
    w = workload("edges7_shelf", n=1400)
    qa, qb = w["qa"], w["qb"]
    counts = orc.edge_n_states_batch(qa, qb, RES).astype(np.int64)
    q, e, _ = _states_of(qa, qb, counts)
    cmin, _ = orc.states(w["robot"], w["env"], q)
    near = np.zeros(len(qa), bool)
    np.logical_or.at(near, e, np.abs(cmin) <= BAND)
    keep = np.flatnonzero(~near)[:1024]
    assert len(keep) == 1024
    sub = np.isin(e, keep)
    visits, want = _replay(counts[keep], (cmin < 0)[sub])
    r, env = vk.Robot(w["robot"]), vk.Env(w["env"])
    flops = torch.zeros(8, dtype=torch.int64, device="cuda")
    got = host(vk.validate_edges_counted(r, env, dev(qa[keep]), dev(qb[keep]), flops,
                                         resolution=RES))
    f = host(flops).astype(np.int64)
    say(f"replay: {len(keep)} edges, {visits.sum()} rake slots (kernel {f[7]}), "
        f"collision rate {want.mean():.3f}; FLOPs total {f[0]:.4e}, method {f[1:5].sum():.4e}, "
        f"re-posing {f[5]:.4e}, surplus lanes {f[6]:.4e}")
    np.testing.assert_array_equal(got, want)
    assert f[7] == visits.sum()
    assert f[0] == f[1:7].sum() and (f[1:7] > 0).all()


def test_surplus_lanes_only_when_the_rake_is_ragged(vk):
    """Edges of exactly 64 or 128 states fill every rake slot: no surplus work.  Edges of 65
    states leave 63 surplus lanes in their second step."""
    import torch
    w = workload("edges7_shelf", n=512)
    r, env = vk.Robot(w["robot"]), vk.Env({})
    qa, qb = dev(w["qa"]), dev(w["qb"])
    for n, surplus in ((64, False), (128, False), (65, True)):
        ns = torch.full((512,), n, dtype=torch.int32, device="cuda")
        flops = torch.zeros(8, dtype=torch.int64, device="cuda")
        vk.validate_edges_counted(r, env, qa, qb, flops, n_states=ns)
        f = host(flops)
        say(f"n = {n}: surplus FLOPs {f[6]}, rake slots {f[7]}")
        assert (f[6] > 0) == surplus
        if n == 128:
            assert f[7] <= 512 * 128
