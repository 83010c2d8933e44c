"""GPU tests of the many-query RRT-Connect: the tree primitives against brute-force numpy
references, and planned paths checked edge by edge with the FP64 oracle."""
import numpy as np
import pytest

from helpers import dev, host, say
from oracle import roadmap
from synthetic import workload, rng, uniform_states

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _trees(Q=37, cap=300, dof=7):
    g = rng("gpu-tree", "trees")
    nodes = g.uniform(-2.9, 2.9, (Q, cap, dof)).astype(np.float32)
    sizes = g.integers(0, cap + 1, Q).astype(np.int32)
    sizes[0], sizes[1], sizes[2] = 0, 1, cap
    nodes[3, 5] = nodes[3, 9]                  # a tie: the lower index must win
    targets = g.uniform(-2.9, 2.9, (Q, dof)).astype(np.float32)
    targets[3] = nodes[3, 9] + np.float32(1e-3)
    return nodes, sizes, targets


def test_tree_nearest_parity(vk):
    nodes, sizes, targets = _trees()
    Q = len(sizes)
    active = np.ones(Q, np.uint8)
    active[7] = 0
    near = host(vk.tree_nearest(dev(nodes), dev(sizes), dev(targets), dev(active)))
    for q in range(Q):
        if sizes[q] == 0 or not active[q]:
            assert near[q] == -1
            continue
        d2 = roadmap.dist2_f32(targets[q:q + 1], nodes[q, :sizes[q]])[0]
        want = int(np.lexsort((np.arange(sizes[q]), d2))[0])
        assert near[q] == want, q
    assert near[3] == 5


def test_tree_steer_and_append(vk):
    import torch
    nodes, sizes, targets = _trees()
    Q, cap, dof = nodes.shape
    sizes = np.maximum(sizes, 1).astype(np.int32)
    sizes[2] = cap                            # a full tree: nothing may be appended
    near = np.array([q % s for q, s in enumerate(sizes)], np.int32)
    step = 0.7
    targets[4] = nodes[4, near[4]] + np.float32(0.1)        # within reach
    qn, reached = vk.tree_steer(dev(nodes), dev(near), dev(targets), step)
    qn, reached = host(qn), host(reached)
    for q in range(Q):
        a = nodes[q, near[q]].astype(np.float64)
        d = targets[q].astype(np.float64) - a
        L = np.linalg.norm(d)
        if L <= step:
            assert reached[q] == 1 and np.array_equal(qn[q], targets[q])
        else:
            assert reached[q] == 0
            np.testing.assert_allclose(qn[q], a + d * step / L, atol=2e-6)
    nd, pr, sz = dev(nodes), torch.full((Q, cap), -1, dtype=torch.int32, device="cuda"), dev(sizes)
    ok = np.ones(Q, np.uint8)
    ok[5] = 0
    added = host(vk.tree_append(nd, pr, sz, dev(qn), dev(near), dev(ok)))
    sz, nd, pr = host(sz), host(nd), host(pr)
    for q in range(Q):
        if not ok[q] or sizes[q] >= cap:
            assert added[q] == -1 and sz[q] == sizes[q]
        else:
            assert added[q] == sizes[q] and sz[q] == sizes[q] + 1
            assert np.array_equal(nd[q, added[q]], qn[q]) and pr[q, added[q]] == near[q]


def _queries(orc, w, n, tag):
    """n start/goal pairs of collision-free states (checked by the oracle)."""
    g = rng("gpu-rrt", tag)
    r = w["robot"]
    out = []
    while len(out) < 2 * n:
        q = uniform_states(g, r["dof"], 256)
        _, flag = orc.states(r, w["env"], q)
        out += [q[:, i] for i in np.nonzero(flag == 0)[0]]
    out = np.asarray(out[:2 * n], np.float32)
    return out[0::2], out[1::2]


def test_rrt_connect_paths_are_valid(vk, orc):
    from paper_2309_14545_amd import planning
    w = workload("edges7_shelf", n=1)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    starts, goals = _queries(orc, w, 48, "q7")
    lo, hi = w["robot"]["q_lo"], w["robot"]["q_hi"]
    res = planning.rrt_connect(r, e, dev(starts), dev(goals), lo, hi, max_iters=300, cap=2048, seed=3)
    say(f"rrt-connect: solved {res['solved'].sum()} of {len(starts)} in {res['iterations']} "
        f"iterations, {res['rounds']} rounds, {res['edges']} edges")
    assert res["solved"].mean() >= 0.5
    for q, path in enumerate(res["paths"]):
        if path is None:
            continue
        np.testing.assert_array_equal(path[0], starts[q])
        np.testing.assert_array_equal(path[-1], goals[q])
        _, cls, _ = orc.edges(w["robot"], w["env"], path[:-1], path[1:], res=RES)
        assert not np.any(cls == 1), q        # no edge collides outside the near-contact band
