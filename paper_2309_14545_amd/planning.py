"""Many-query RRT-Connect on the GPU primitives (the RRT-Connect planner of Sec. III-E).

RRT-Connect grows one tree from the start and one from the goal.  Each iteration samples a
configuration, extends one tree toward it by at most `step`, then repeatedly extends the other
tree toward the new node until it reaches it or an edge collides; the trees swap roles every
iteration.  Here one iteration does this for every unsolved query at once: nearest nodes,
steering and appends are kernels over the queries (vk_tree_*), and each extension round checks
all of its edges with one validate_edges launch, at the same resolution as every other edge.
The loop itself, a handful of launches per round, runs on the host; samples come from a seeded
torch generator on the device.
"""
from __future__ import annotations

import numpy as np

from . import tree_append, tree_nearest, tree_steer, validate_edges


def rrt_connect(robot, env, starts, goals, q_lo, q_hi, step: float = 0.6,
                max_iters: int = 500, max_connect: int = 16, cap: int = 4096, seed: int = 0,
                resolution: float = 1.0 / 32.0):
    """Plan for Q queries at once.  starts, goals: [Q, dof] collision-free configurations (CUDA
    float32); q_lo, q_hi: [dof] sampling bounds.  Returns a dict with `solved` (bool [Q]),
    `paths` (a list of [n_i, dof] numpy arrays, None for unsolved queries), `iterations`,
    `rounds` (extension rounds, one edge batch each) and `edges` (edges checked)."""
    import torch
    dev = starts.device
    Q, dof = starts.shape
    nodes = torch.zeros((2, Q, cap, dof), dtype=torch.float32, device=dev)
    parents = torch.full((2, Q, cap), -1, dtype=torch.int32, device=dev)
    sizes = torch.ones((2, Q), dtype=torch.int32, device=dev)
    nodes[0, :, 0] = starts
    nodes[1, :, 0] = goals
    solved = torch.zeros(Q, dtype=torch.bool, device=dev)
    meet = torch.full((2, Q), -1, dtype=torch.int64, device=dev)    # meeting node per tree
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    lo = torch.as_tensor(np.asarray(q_lo, np.float32), device=dev)
    span = torch.as_tensor(np.asarray(q_hi, np.float32), device=dev) - lo
    rounds = 0
    it = 0

    rows = torch.arange(Q, device=dev)
    edge_count = torch.zeros((), dtype=torch.int64, device=dev)

    def extend(t, target, active):
        """One extension of tree t toward target[q] for the active queries.  Every row's edge is
        checked in one batch (an inactive row's edge has length zero, two states) so that no
        host synchronisation is needed to pick the active rows."""
        nonlocal rounds
        near = tree_nearest(nodes[t], sizes[t], target, active.to(torch.uint8))
        qnew, reached = tree_steer(nodes[t], near, target, step)
        qnear = nodes[t][rows, near.clamp(min=0).long()]
        qnew = torch.where(active[:, None], qnew, qnear).contiguous()
        flags = validate_edges(robot, env, qnear, qnew, resolution=resolution)
        rounds += 1
        edge_count.add_(active.sum())
        ok = active & (flags == 0) & (near >= 0)
        added = tree_append(nodes[t], parents[t], sizes[t], qnew, near, ok.to(torch.uint8))
        return qnew, reached.bool(), added

    a = 0
    for it in range(1, max_iters + 1):
        active = ~solved
        if not bool(active.any()):
            it -= 1
            break
        q_rand = lo + span * torch.rand((Q, dof), generator=gen, device=dev)
        q_new, _, added = extend(a, q_rand, active)
        b = 1 - a
        target = q_new
        going = added >= 0
        for _ in range(max_connect):
            if not bool(going.any()):
                break
            _, reached, addb = extend(b, target, going)
            hit = going & (addb >= 0) & reached
            meet[a] = torch.where(hit, added.long(), meet[a])
            meet[b] = torch.where(hit, addb.long(), meet[b])
            solved |= hit
            going = going & (addb >= 0) & ~reached
        a = b

    edges = int(edge_count.item())
    # paths, on the host: root of tree 0 .. meeting node, then tree 1's meeting node .. root
    sol = solved.cpu().numpy()
    nd = nodes.cpu().numpy()
    par = parents.cpu().numpy()
    mt = meet.cpu().numpy()
    paths = []
    for q in range(Q):
        if not sol[q]:
            paths.append(None)
            continue
        half = []
        for t in (0, 1):
            chain, v = [], int(mt[t, q])
            while v >= 0:
                chain.append(nd[t, q, v])
                v = int(par[t, q, v])
            half.append(chain)
        # tree 0's chain runs meet -> start; tree 1's meet -> goal; both meet nodes are equal
        path = half[0][::-1] + half[1][1:]
        paths.append(np.asarray(path, np.float32))
    return {"solved": sol, "paths": paths, "iterations": it, "rounds": rounds, "edges": edges}
