"""GPU tests of the many-query RRT-Connect: the tree primitives against brute-force numpy
references, and planned paths checked edge by edge with the FP64 oracle."""
import numpy as np
import pytest

from helpers import dev, host, say, nearest_against_exact
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
    ties = 0
    for q in range(Q):
        if sizes[q] == 0 or not active[q]:
            assert near[q] == -1
            continue
        # the FP64 definition (near ties within the FP32 rounding bound reported) ...
        ties += nearest_against_exact(targets[q], nodes[q, :sizes[q]], int(near[q]))
        # ... and the fixed-order FP32 evaluation, bit for bit
        d2 = roadmap.dist2_f32(targets[q:q + 1], nodes[q, :sizes[q]])[0]
        want = int(np.lexsort((np.arange(sizes[q]), d2))[0])
        assert near[q] == want, q
    say(f"tree nearest: {Q} queries, {ties} near ties")
    assert near[3] == 5                        # identical nodes: the lower index


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


def test_rrt_extend_matches_the_primitives(vk):
    """The fused extension gives the nearest node, step and reach flag of tree_nearest and
    tree_steer bit for bit, and the edge starts at the nearest node."""
    import torch
    nodes, sizes, targets = _trees()
    Q, cap, dof = nodes.shape
    g = rng("gpu-tree", "extend")
    active = (g.random(Q) < 0.8).astype(np.uint8)
    active[:3] = 1                              # the empty, one-node and full trees are active
    nd, sz, tg, ac = dev(nodes), dev(sizes), dev(targets), dev(active)
    step = 0.7
    f32 = dict(dtype=torch.float32, device="cuda")
    qnear, qnew = torch.full((Q, dof), np.nan, **f32), torch.full((Q, dof), np.nan, **f32)
    near = torch.full((Q,), -7, dtype=torch.int32, device="cuda")
    reached = torch.full((Q,), 9, dtype=torch.uint8, device="cuda")
    vk.rrt_extend(nd, sz, tg, ac, step, qnear, qnew, near, reached)
    want_near = host(vk.tree_nearest(nd, sz, tg, ac))
    want_qnew, want_reached = map(host, vk.tree_steer(nd, dev(want_near), tg, step))
    near, reached, qnear, qnew = host(near), host(reached), host(qnear), host(qnew)
    np.testing.assert_array_equal(near, want_near)
    for q in range(Q):
        if near[q] < 0:
            root = nodes[q, 0] if sizes[q] > 0 else targets[q]
            assert reached[q] == 0, q
            np.testing.assert_array_equal(qnear[q], root)
            np.testing.assert_array_equal(qnew[q], root)
        else:
            assert reached[q] == want_reached[q], q
            np.testing.assert_array_equal(qnear[q], nodes[q, near[q]])
            np.testing.assert_array_equal(qnew[q], want_qnew[q])
    assert near[0] == -1 and near[3] == 5


def _commit_model(nodes, parents, sizes, qnew, near, reached, flags, going, edges,
                  from_added=None, meet_this=None, meet_from=None, solved=None):
    """The bookkeeping of vk_rrt_commit written out per query."""
    Q, cap, _ = nodes.shape
    added = np.full(Q, -1, np.int32)
    for q in range(Q):
        if not going[q]:
            continue
        edges += 1
        s, n = sizes[q], near[q]
        if flags[q] == 0 and 0 <= n < s and s < cap:
            nodes[q, s], parents[q, s], sizes[q], added[q] = qnew[q], n, s + 1, s
    if from_added is None:
        going[:] = added >= 0
    else:
        at = (added >= 0) & (reached != 0)
        meet_this[at], meet_from[at], solved[at] = added[at], from_added[at], 1
        going[:] = (added >= 0) & (reached == 0)
    return added, edges


@pytest.mark.parametrize("connect", [False, True])
def test_rrt_commit_bookkeeping(vk, connect):
    import torch
    nodes, sizes, _ = _trees()
    Q, cap, dof = nodes.shape
    g = rng("gpu-tree", f"commit-{connect}")
    parents = g.integers(-1, cap, (Q, cap)).astype(np.int32)
    qnew = g.uniform(-3, 3, (Q, dof)).astype(np.float32)
    near = (g.integers(-1, cap, Q)).astype(np.int32)
    near[:8] = np.minimum(sizes[:8], 1) - 1     # valid where the tree has a node
    reached = (g.random(Q) < 0.5).astype(np.uint8)
    flags = (g.random(Q) < 0.3).astype(np.uint8)
    going = (g.random(Q) < 0.8).astype(np.uint8)
    from_added = g.integers(-1, cap, Q).astype(np.int32)
    meet = np.full((2, Q), -1, np.int64)
    solved = np.zeros(Q, np.uint8)
    d = [dev(x) for x in (nodes, parents, sizes, qnew, near, reached, flags, going)]
    added = torch.full((Q,), 77, dtype=torch.int32, device="cuda")
    edges = torch.tensor([5], dtype=torch.int64, device="cuda")
    dmeet, dsolved, dfrom = dev(meet), dev(solved), dev(from_added)
    if connect:
        vk.rrt_commit(*d, added, edges, from_added=dfrom, meet_this=dmeet[1], meet_from=dmeet[0],
                      solved=dsolved)
    else:
        vk.rrt_commit(*d, added, edges)
    want_added, want_edges = _commit_model(nodes, parents, sizes, qnew, near, reached, flags, going,
                                           5, *((from_added, meet[1], meet[0], solved)
                                                if connect else ()))
    np.testing.assert_array_equal(host(added), want_added)
    assert int(host(edges)[0]) == want_edges
    for got, want in zip([host(x) for x in (d[0], d[1], d[2], d[7], dmeet, dsolved)],
                         (nodes, parents, sizes, going, meet, solved)):
        np.testing.assert_array_equal(got, want)
    assert (want_added >= 0).any() and (want_added < 0).any()
    if connect:
        assert solved.any()


def _rrt_by_primitives(vk, r, e, starts, goals, q_lo, q_hi, step=0.6, max_iters=500,
                       max_connect=16, cap=4096, seed=0, resolution=RES):
    """RRT-Connect composed from the separate tree primitives, validate_edges and torch glue,
    with the same sampling sequence as planning.rrt_connect."""
    import torch
    Q, dof = starts.shape
    nodes = torch.zeros((2, Q, cap, dof), dtype=torch.float32, device="cuda")
    parents = torch.full((2, Q, cap), -1, dtype=torch.int32, device="cuda")
    sizes = torch.ones((2, Q), dtype=torch.int32, device="cuda")
    nodes[0, :, 0], nodes[1, :, 0] = starts, goals
    solved = torch.zeros(Q, dtype=torch.bool, device="cuda")
    meet = torch.full((2, Q), -1, dtype=torch.int64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    lo = torch.as_tensor(np.asarray(q_lo, np.float32), device="cuda")
    span = torch.as_tensor(np.asarray(q_hi, np.float32), device="cuda") - lo
    rows = torch.arange(Q, device="cuda")
    count = {"rounds": 0, "edges": 0}

    def extend(t, target, active):
        near = vk.tree_nearest(nodes[t], sizes[t], target, active.to(torch.uint8))
        qn, reached = vk.tree_steer(nodes[t], near, target, step)
        qnear = nodes[t][rows, near.clamp(min=0).long()]
        qn = torch.where(active[:, None], qn, qnear).contiguous()
        flags = vk.validate_edges(r, e, qnear, qn, resolution=resolution)
        count["rounds"] += 1
        count["edges"] += int(active.sum())
        ok = active & (flags == 0) & (near >= 0)
        added = vk.tree_append(nodes[t], parents[t], sizes[t], qn, near, ok.to(torch.uint8))
        return qn, reached.bool(), added

    a, it = 0, 0
    for it in range(1, max_iters + 1):
        active = ~solved
        if not bool(active.any()):
            it -= 1
            break
        q_rand = lo + span * torch.rand((Q, dof), generator=gen, device="cuda")
        q_new, _, added = extend(a, q_rand, active)
        b = 1 - a
        going = added >= 0
        for _ in range(max_connect):
            if not bool(going.any()):
                break
            _, reached, addb = extend(b, q_new, going)
            hit = going & (addb >= 0) & reached
            meet[a] = torch.where(hit, added.long(), meet[a])
            meet[b] = torch.where(hit, addb.long(), meet[b])
            solved |= hit
            going = going & (addb >= 0) & ~reached
        a = b
    return dict(solved=host(solved), meet=host(meet), nodes=host(nodes), parents=host(parents),
                iterations=it, **count)


@pytest.mark.parametrize("graphs", [True, False], ids=["graphs", "direct"])
def test_rrt_connect_matches_the_primitive_loop(vk, orc, graphs):
    """The fused planner takes exactly the steps of the loop composed from the primitives: the
    same solved queries, iterations, rounds, edges and paths, whether its rounds are replayed
    from HIP graphs (with the host's checks and sampling between replays) or launched
    directly."""
    from paper_2309_14545_amd import planning
    w = workload("edges7_shelf", n=1)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    starts, goals = _queries(orc, w, 40, "q7-same")
    lo, hi = w["robot"]["q_lo"], w["robot"]["q_hi"]
    kw = dict(max_iters=60, cap=512, seed=11)
    res = planning.rrt_connect(r, e, dev(starts), dev(goals), lo, hi, graphs=graphs, **kw)
    ref = _rrt_by_primitives(vk, r, e, dev(starts), dev(goals), lo, hi, **kw)
    say(f"fused rrt-connect: solved {res['solved'].sum()} of {len(starts)}, {res['iterations']} "
        f"iterations, {res['rounds']} rounds, {res['edges']} edges")
    np.testing.assert_array_equal(res["solved"], ref["solved"])
    for k in ("iterations", "rounds", "edges"):
        assert res[k] == ref[k], k
    assert 0 < res["solved"].sum()
    for q, path in enumerate(res["paths"]):
        if path is None:
            assert not ref["solved"][q]
            continue
        half = []
        for t in (0, 1):
            chain, v = [], int(ref["meet"][t, q])
            while v >= 0:
                chain.append(ref["nodes"][t, q, v])
                v = int(ref["parents"][t, q, v])
            half.append(chain)
        np.testing.assert_array_equal(path, np.asarray(half[0][::-1] + half[1][1:], np.float32))
