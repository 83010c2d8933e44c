"""Randomized shortcutting (the path simplification of Sec. III-E) round by round against a
plain reference: the proposals from the same random words, the candidate flags against the FP64
oracle's edge classes (a near-contact candidate takes the kernel's flag: either answer is
right there), and the spliced paths against the reference splice of those flags.  Every
accepted shortcut is free per the oracle, endpoints stay, paths only lose waypoints and their
length never grows."""
import numpy as np
import pytest

from helpers import dev, host, say, edge_mismatches
from synthetic import workload

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def ref_propose(lens, M, k, rnd):
    P = len(lens)
    pairs = np.full((P * k, 2), -1, np.int64)
    for p in range(P):
        n = int(lens[p])
        for c in range(k):
            s = p * k + c
            if n >= 3:
                i = int(rnd[2 * s]) % (n - 2)
                j = i + 2 + int(rnd[2 * s + 1]) % (n - i - 2)
                pairs[s] = (p * M + i, p * M + j)
    return pairs


def ref_apply(paths, lens, k, pairs, flags):
    P, M, _ = paths.shape
    paths, lens = paths.copy(), lens.copy()
    taken = np.zeros(P, np.uint8)
    for p in range(P):
        best = None
        for c in range(k):
            a, b = pairs[p * k + c]
            if a < 0 or flags[p * k + c]:
                continue
            i, j = a - p * M, b - p * M
            if best is None or j - i > best[1] - best[0]:
                best = (i, j)
        if best is not None:
            i, j = best
            n = lens[p]
            keep = np.concatenate([paths[p, :i + 1], paths[p, j:n]])
            paths[p, :len(keep)] = keep
            lens[p] = len(keep)
            taken[p] = 1
    return paths, lens, taken


def _lengths(paths, lens):
    w = paths.astype(np.float64)
    return np.array([np.linalg.norm(np.diff(w[p, :lens[p]], axis=0), axis=1).sum()
                     for p in range(len(lens))])


def test_shortcut_rounds_against_the_reference(vk, orc):
    import torch
    w = workload("shortcut7_shelf", n=256)
    robot, env = w["robot"], w["env"]
    r, e = vk.Robot(robot), vk.Env(env)
    P, M, dof, k = 256, 32, 7, 4
    paths = w["nodes"].reshape(P, M, dof).copy()
    g = np.random.default_rng(3)
    lens = g.integers(2, M + 1, P).astype(np.int32)      # ragged paths, some too short to cut
    lens[:3] = (0, 1, 2)
    paths_d, lens_d = dev(paths), dev(lens)
    start_len = _lengths(paths, lens)
    first, last = paths[np.arange(P), 0].copy(), paths[np.arange(P), np.maximum(lens - 1, 0)].copy()
    total_taken = 0
    for rnd_i in range(8):
        rnd = g.integers(0, 2 ** 32, 2 * P * k, dtype=np.uint64).astype(np.uint32)
        pairs_ref = ref_propose(lens, M, k, rnd)
        pairs = vk.shortcut_propose(lens_d, M, k, dev(rnd.view(np.int32)))
        np.testing.assert_array_equal(host(pairs), pairs_ref)
        flags = host(vk.validate_edges_indexed(r, e, paths_d.view(P * M, dof), pairs,
                                               resolution=RES))
        real = pairs_ref[:, 0] >= 0
        nodes = paths.reshape(P * M, dof)
        _, cls, _ = orc.edges(robot, env, nodes[pairs_ref[real, 0]], nodes[pairs_ref[real, 1]],
                              res=RES)
        bad, near = edge_mismatches(flags[real], cls)
        assert bad == 0
        ref_flags = np.zeros(P * k, np.uint8)
        ref_flags[real] = np.where(cls == 2, flags[real], cls == 1)
        accepted = torch.empty(P, dtype=torch.uint8, device="cuda")
        vk.shortcut_apply(paths_d, lens_d, k, pairs, dev(flags), accepted)
        paths, lens, taken = ref_apply(paths, lens, k, pairs_ref, ref_flags)
        np.testing.assert_array_equal(host(lens_d), lens)
        got = host(paths_d)
        for p in range(P):
            np.testing.assert_array_equal(got[p, :lens[p]], paths[p, :lens[p]])
        np.testing.assert_array_equal(host(accepted), taken)
        total_taken += int(taken.sum())
        say(f"round {rnd_i}: {int(real.sum())} candidates, {near} near contact, "
            f"{int(taken.sum())} shortcuts")
    assert total_taken > 0
    # every accepted shortcut is free: each output edge is either an original path edge or an
    # edge the oracle does not find colliding; lengths never grow; endpoints stay
    end_len = _lengths(paths, lens)
    assert np.all(end_len <= start_len * (1 + 1e-6) + 1e-9)
    keep = lens >= 1
    np.testing.assert_array_equal(paths[keep, 0], first[keep])
    np.testing.assert_array_equal(paths[np.arange(P)[keep], lens[keep] - 1], last[keep])
    say(f"shortcut: {total_taken} shortcuts over 8 rounds; mean length "
        f"{start_len.mean():.3f} -> {end_len.mean():.3f}")


def test_shortcut_loop_on_planner_paths(vk, orc):
    """planning.shortcut on RRT-Connect paths in the shelf scene: every output edge free per the
    oracle (outside the band), lengths never grow, endpoints stay."""
    import torch
    from paper_2309_14545_amd import planning
    from synthetic import rng, uniform_states
    w = workload("edges7_shelf", n=1)
    robot, env = w["robot"], w["env"]
    r, e = vk.Robot(robot), vk.Env(env)
    q = uniform_states(rng("gpu-shortcut", "queries"), 7, 4096)
    cmin, _ = orc.states(robot, env, q)
    free = q[:, cmin > 1e-3].T[:128]
    starts, goals = dev(np.ascontiguousarray(free[0::2])), dev(np.ascontiguousarray(free[1::2]))
    res = planning.rrt_connect(r, e, starts, goals, robot["q_lo"], robot["q_hi"], max_iters=200,
                               cap=1024, seed=2)
    paths = [p for p in res["paths"] if p is not None]
    assert len(paths) >= 48
    P = len(paths)
    pd, ld = planning.pack_paths(paths, 7)
    before = planning.path_lengths(pd, ld)
    out = planning.shortcut(r, e, pd, ld, rounds=24, k=8, seed=5)
    after = planning.path_lengths(pd, ld)
    w_out, l_out = host(pd), host(ld)
    a = np.concatenate([w_out[p, :l_out[p] - 1] for p in range(P)])
    b = np.concatenate([w_out[p, 1:l_out[p]] for p in range(P)])
    _, cls, _ = orc.edges(robot, env, a, b, res=RES)
    say(f"planner paths: {P}, {out['accepted']} shortcuts, length {before.mean():.3f} -> "
        f"{after.mean():.3f}, output edges {len(a)}, colliding {int((cls == 1).sum())}, "
        f"near {int((cls == 2).sum())}")
    assert (cls != 1).all()
    assert np.all(after <= before * (1 + 1e-6) + 1e-9) and after.mean() < 0.9 * before.mean()
    for p in range(P):
        np.testing.assert_array_equal(w_out[p, 0], paths[p][0])
        np.testing.assert_array_equal(w_out[p, l_out[p] - 1], paths[p][-1])
