"""Many-query RRT-Connect and randomized shortcutting on the GPU primitives (the planner and
path simplification of Sec. III-E).

RRT-Connect grows one tree from the start and one from the goal.  Each iteration samples a
configuration, extends one tree toward it by at most `step`, then repeatedly extends the other
tree toward the new node until it reaches it or an edge collides; the trees swap roles every
iteration.  Here one iteration does this for every unsolved query at once.  An extension round
is three launches over all queries: rrt_extend (nearest node, step, the edge to check),
validate_edges (every query's edge in one launch, at the same resolution as every other edge)
and rrt_commit (appends, the meeting nodes, which queries go on), followed by one host check of
whether any query goes on.  The four kinds of round (either tree, toward the sample or toward
the other tree's new node) are captured once as HIP graphs over fixed buffers and replayed.
Samples come from a seeded torch generator on the device.
"""
from __future__ import annotations

import numpy as np

from . import (reserve, rrt_commit, rrt_extend, shortcut_apply, shortcut_propose, validate_edges,
               validate_edges_indexed)


def rrt_connect(robot, env, starts, goals, q_lo, q_hi, step: float = 0.6,
                max_iters: int = 500, max_connect: int = 16, cap: int = 4096, seed: int = 0,
                resolution: float = 1.0 / 32.0, graphs: bool = True):
    """Plan for Q queries at once.  starts, goals: [Q, dof] collision-free configurations (CUDA
    float32); q_lo, q_hi: [dof] sampling bounds.  Returns a dict with `solved` (bool [Q]),
    `paths` (a list of [n_i, dof] numpy arrays, None for unsolved queries), `iterations`,
    `rounds` (extension rounds, one edge batch each) and `edges` (edges checked).  With
    graphs=False every round is launched directly instead of replayed from a HIP graph (the
    same kernels on the same buffers)."""
    import torch
    dev = starts.device
    Q, dof = starts.shape
    nodes = torch.zeros((2, Q, cap, dof), dtype=torch.float32, device=dev)
    parents = torch.full((2, Q, cap), -1, dtype=torch.int32, device=dev)
    sizes = torch.ones((2, Q), dtype=torch.int32, device=dev)
    nodes[0, :, 0] = starts
    nodes[1, :, 0] = goals
    solved = torch.zeros(Q, dtype=torch.uint8, device=dev)
    meet = torch.full((2, Q), -1, dtype=torch.int64, device=dev)    # meeting node per tree
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    lo = torch.as_tensor(np.asarray(q_lo, np.float32), device=dev)
    span = torch.as_tensor(np.asarray(q_hi, np.float32), device=dev) - lo
    edge_count = torch.zeros(1, dtype=torch.int64, device=dev)
    # per-round buffers, one set per role: [0] the extension toward the sample, [1] the connects
    f32 = dict(dtype=torch.float32, device=dev)
    qnear = torch.empty((2, Q, dof), **f32)
    qnew = torch.empty((2, Q, dof), **f32)
    near = torch.empty((2, Q), dtype=torch.int32, device=dev)
    reached = torch.empty((2, Q), dtype=torch.uint8, device=dev)
    added = torch.empty((2, Q), dtype=torch.int32, device=dev)
    flags = torch.empty(Q, dtype=torch.uint8, device=dev)
    going = torch.empty(Q, dtype=torch.uint8, device=dev)
    q_rand = torch.empty((Q, dof), **f32)
    rounds = 0
    it = 0

    def launch(t, r):
        """One extension round of tree t: toward the sample (r = 0) or toward the node the other
        tree added this iteration (r = 1)."""
        connect = r == 1
        rrt_extend(nodes[t], sizes[t], qnew[0] if connect else q_rand, going, step, qnear[r],
                   qnew[r], near[r], reached[r])
        validate_edges(robot, env, qnear[r], qnew[r], resolution=resolution, out=flags)
        rrt_commit(nodes[t], parents[t], sizes[t], qnew[r], near[r], reached[r], flags, going,
                   added[r], edge_count, from_added=added[0] if connect else None,
                   meet_this=meet[t] if connect else None,
                   meet_from=meet[1 - t] if connect else None, solved=solved)

    run = launch
    if graphs:
        side = torch.cuda.Stream(device=dev)
        reserve(stream=side)              # the edge launch's work-queue counters on that stream
        captured = {}
        for t in (0, 1):
            for r in (0, 1):
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                    launch(t, r)
                captured[(t, r)] = g
        run = lambda t, r: captured[(t, r)].replay()   # noqa: E731

    a = 0
    for it in range(1, max_iters + 1):
        torch.eq(solved, 0, out=going)
        if not bool(going.any()):
            it -= 1
            break
        torch.rand((Q, dof), generator=gen, device=dev, out=q_rand)
        q_rand.mul_(span).add_(lo)
        run(a, 0)
        rounds += 1
        b = 1 - a
        for _ in range(max_connect):
            if not bool(going.any()):
                break
            run(b, 1)
            rounds += 1
        a = b

    edges = int(edge_count.item())
    # paths, on the host: root of tree 0 .. meeting node, then tree 1's meeting node .. root
    sol = solved.cpu().numpy().astype(bool)
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


def pack_paths(paths, dof: int, device="cuda"):
    """Pack a list of [n_i, dof] waypoint arrays into (paths [P, M, dof], lens [P]) tensors."""
    import torch
    P = len(paths)
    M = max(len(p) for p in paths)
    buf = np.zeros((P, M, dof), np.float32)
    lens = np.zeros(P, np.int32)
    for i, p in enumerate(paths):
        buf[i, :len(p)] = p
        lens[i] = len(p)
    return torch.from_numpy(buf).to(device), torch.from_numpy(lens).to(device)


def path_lengths(paths, lens):
    """Euclidean joint-space length of each packed path (FP64, on the host)."""
    P = paths.shape[0]
    w = paths.detach().cpu().numpy().astype(np.float64)
    n = lens.cpu().numpy()
    return np.array([np.linalg.norm(np.diff(w[p, :n[p]], axis=0), axis=1).sum() for p in range(P)])


def shortcut(robot, env, paths, lens, rounds: int = 64, k: int = 8, seed: int = 0,
             resolution: float = 1.0 / 32.0):
    """Randomized shortcutting of P paths at once, in place: paths [P, M, dof] (CUDA float32),
    lens [P] (CUDA int32).  Each round proposes k waypoint pairs per path, validates all P * k
    straight edges in one launch and splices in, per path, the valid one that skips the most
    waypoints (vk_shortcut_*).  The random words of every round are drawn up front from a seeded
    torch generator on the device.  Returns {"rounds", "accepted" (shortcuts taken),
    "edges_checked"}."""
    import torch
    P, M, dof = paths.shape
    dev = paths.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    rnd = torch.randint(0, 2 ** 31 - 1, (rounds, 2 * P * k), generator=gen, device=dev,
                        dtype=torch.int32)
    nodes = paths.view(P * M, dof)
    pairs = torch.empty((P * k, 2), dtype=torch.int32, device=dev)
    flags = torch.empty(P * k, dtype=torch.uint8, device=dev)
    accepted = torch.empty((rounds, P), dtype=torch.uint8, device=dev)
    for r in range(rounds):
        shortcut_propose(lens, M, k, rnd[r], pairs)
        validate_edges_indexed(robot, env, nodes, pairs, resolution=resolution, out=flags)
        shortcut_apply(paths, lens, k, pairs, flags, accepted[r])
    return {"rounds": rounds, "accepted": int(accepted.sum().item()), "edges_checked": rounds * P * k}
