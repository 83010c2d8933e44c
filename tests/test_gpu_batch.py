"""GPU parity of the mixed-robot edge batch (persistent launch replayed from a HIP graph)."""
import numpy as np
import pytest

from helpers import dev, host, say, edge_mismatches
from synthetic import workload, pack_edge_sets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def _pack(vk, w, max_edges=None):
    robots = [vk.Robot(r) for r in w["robots"]]
    envs = [vk.Env(e) for e in w["envs"]]
    qa, qb, sets, total = pack_edge_sets(w, max_edges)
    return robots, envs, sets, dev(qa), dev(qb), total


def test_batch_parity_and_replays(vk, orc):
    import torch
    w = workload("mixed", n=24)
    robots, envs, sets, qa, qb, total = _pack(vk, w, max_edges=60)
    out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    say("edge batch sets", len(sets), "edges", total)
    batch = vk.EdgeBatch(robots, envs, sets)
    results = []
    for rep in range(3):
        out.fill_(7)
        batch.run(qa, qb, out)
        results.append(host(out).copy())
        # eager work between replays
        torch.cuda.synchronize()
        _ = (qa * 2).sum().item()
    for r in results[1:]:
        np.testing.assert_array_equal(r, results[0])
    flags = results[0]
    assert set(np.unique(flags)) <= {0, 1}
    qa_h, qb_h = host(qa), host(qb)
    bad_total, near_total = 0, 0
    for (ri, ei, off, ne, oo) in sets:
        dof = w["robots"][ri]["dof"]
        a = qa_h[off:off + ne * dof].reshape(ne, dof)
        b = qb_h[off:off + ne * dof].reshape(ne, dof)
        _, cls, _ = orc.edges(w["robots"][ri], w["envs"][ei], a, b)
        bad, near = edge_mismatches(flags[oo:oo + ne], cls)
        bad_total += bad
        near_total += near
        # same flags as the single-robot batched call
        single = host(vk.validate_edges(robots[ri], envs[ei], dev(a), dev(b)))
        np.testing.assert_array_equal(single, flags[oo:oo + ne])
    say(f"  mismatches outside band {bad_total}, near-contact {near_total}")
    assert bad_total == 0


def test_batch_new_arrays_each_run(vk):
    """One batch replayed on other arrays: every run validates the edges and writes the flags of
    the arrays it is given (the graph's launch is re-pointed), alternating between two sets of
    endpoints and two flag buffers, with eager work between runs."""
    import torch
    w = workload("mixed", n=16)
    robots, envs, sets, qa, qb, total = _pack(vk, w, max_edges=50)
    # the second endpoints: each edge cut to its first twentieth (mostly free where the full
    # edges mostly collide), in new buffers
    qa2, qb2 = qa.clone(), qa + 0.05 * (qb - qa)
    batch = vk.EdgeBatch(robots, envs, sets)
    outs = [torch.full((total,), 7, dtype=torch.uint8, device="cuda") for _ in range(2)]
    want = []
    for a, b in ((qa, qb), (qa2, qb2)):
        flags = np.zeros(total, np.uint8)
        ah, bh = host(a), host(b)
        for (ri, ei, off, ne, oo) in sets:
            dof = w["robots"][ri]["dof"]
            flags[oo:oo + ne] = host(vk.validate_edges(
                robots[ri], envs[ei], dev(ah[off:off + ne * dof].reshape(ne, dof)),
                dev(bh[off:off + ne * dof].reshape(ne, dof))))
        want.append(flags)
    say("new-arrays batch: collision rates", want[0].mean(), want[1].mean())
    assert not np.array_equal(want[0], want[1])
    for rep in range(4):
        k = rep % 2
        outs[k].fill_(7)
        batch.run(*((qa, qb) if k == 0 else (qa2, qb2)), outs[k])
        np.testing.assert_array_equal(host(outs[k]), want[k])
        _ = (qa * 2).sum().item()


def test_empty_batch(vk):
    import torch
    w = workload("mixed", n=2)
    robots = [vk.Robot(r) for r in w["robots"]]
    envs = [vk.Env(e) for e in w["envs"]]
    out = torch.zeros(1, dtype=torch.uint8, device="cuda")
    z = torch.zeros(1, device="cuda")
    b = vk.EdgeBatch(robots, envs, [])
    b.run(z, z, out)
    torch.cuda.synchronize()


def test_batch_with_limit_robots(vk, orc):
    """A mixed batch whose robots span the description's limits (the 7-DoF arm, a robot with a
    19-sphere link and an empty link, 32- and 64-joint chains), each against the shelf and
    against nothing: the batch sizes its workgroups for the largest walk cache.  Flags against
    the oracle and equal to each robot's own validate_edges call."""
    import torch
    from test_gpu_limits import AMPLITUDE, CASES, _env, _robot
    from synthetic import rng
    descs = [workload("edges7_shelf", n=1)["robot"]] + [_robot(n, **CASES[n]) for n in CASES]
    amps = [2.9] + [AMPLITUDE[n] for n in CASES]
    env_descs = [_env(), {}]
    g = rng("gpu-batch", "limits")
    w = {"sets": [], "qa": [], "qb": []}
    for ri, (d, amp) in enumerate(zip(descs, amps)):
        for ei in range(len(env_descs)):
            a = g.uniform(-amp, amp, (40, d["dof"])).astype(np.float32)
            b = (a + g.uniform(-0.8, 0.8, a.shape)).astype(np.float32)
            w["sets"].append((ri, ei, None))
            w["qa"].append(a)
            w["qb"].append(b)
    robots = [vk.Robot(d) for d in descs]
    envs = [vk.Env(e) for e in env_descs]
    qa, qb, sets, total = pack_edge_sets(w)
    qa_d, qb_d = dev(qa), dev(qb)
    out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    batch = vk.EdgeBatch(robots, envs, sets)
    batch.run(qa_d, qb_d, out)
    flags = host(out).copy()
    batch.run(qa_d, qb_d, out)                   # a second replay gives the same flags
    np.testing.assert_array_equal(host(out), flags)
    bad_total = 0
    for k, (ri, ei, off, ne, oo) in enumerate(sets):
        a, b = w["qa"][k], w["qb"][k]
        _, cls, _ = orc.edges(descs[ri], env_descs[ei], a, b)
        bad_total += edge_mismatches(flags[oo:oo + ne], cls)[0]
        single = host(vk.validate_edges(robots[ri], envs[ei], dev(a), dev(b)))
        np.testing.assert_array_equal(single, flags[oo:oo + ne])
    say(f"limit-robot batch: {len(sets)} sets, {total} edges, collision rate {flags.mean():.3f}, "
        f"mismatches {bad_total}")
    assert bad_total == 0 and 0.0 < flags.mean() < 1.0


def test_batch_full_size_sampled(vk, orc):
    """The full mixed batch the benchmark times (1,024 sets over the 7-, 8- and 14-DoF robots,
    about 93 k edges), in the launch shape the autotuner picks for it, replayed twice; the oracle
    checks a seeded sample of 400 edges across the sets."""
    import torch
    from paper_2309_14545_amd import autotune
    w = workload("mixed")
    robots = [vk.Robot(r) for r in w["robots"]]
    envs = [vk.Env(e) for e in w["envs"]]
    qa_h, qb_h, sets, total = pack_edge_sets(w)
    qa, qb = dev(qa_h), dev(qb_h)
    out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    batch, tuned = autotune.tune_batch(robots, envs, sets, qa, qb, out)
    assert batch.launch() == (tuned["block"], tuned["per_cu"])
    say(f"mixed batch full size: {len(sets)} sets, {total} edges, launch {tuned}")
    out.fill_(7)
    batch.run(qa, qb, out)
    flags = host(out).copy()
    batch.run(qa, qb, out)
    np.testing.assert_array_equal(host(out), flags)
    assert set(np.unique(flags)) <= {0, 1}
    g = np.random.default_rng(17)
    owner = np.concatenate([np.full(ne, k) for k, (_, _, _, ne, _) in enumerate(sets)])
    pick = np.sort(g.choice(total, 400, replace=False))
    bad_total = 0
    for k in np.unique(owner[pick]):
        ri, ei, off, ne, oo = sets[k]
        dof = w["robots"][ri]["dof"]
        rows = pick[owner[pick] == k] - oo
        a = qa_h[off:off + ne * dof].reshape(ne, dof)[rows]
        b = qb_h[off:off + ne * dof].reshape(ne, dof)[rows]
        _, cls, _ = orc.edges(w["robots"][ri], w["envs"][ei], a, b)
        bad_total += edge_mismatches(flags[oo + rows], cls)[0]
    say(f"  sampled 400 edges from {len(np.unique(owner[pick]))} sets: mismatches {bad_total}, "
        f"collision rate {flags.mean():.3f}")
    assert bad_total == 0
