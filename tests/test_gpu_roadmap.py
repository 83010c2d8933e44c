"""GPU parity of the roadmap path (k nearest neighbours, undirected pair list, edges given by
node index pairs).  Neighbour lists are checked against the FP64 definition in oracle/roadmap.py
(exact Euclidean distance, near ties within the FP32 rounding bound reported) and, as a
determinism check, bit for bit against the fixed-order FP32 evaluation; edges against the FP64
edge oracle."""
import numpy as np
import pytest

from helpers import dev, host, say, edge_mismatches, knn_against_exact
from oracle import roadmap
from synthetic import workload, rng

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


@pytest.mark.parametrize("n,dim,k", [(1, 7, 3), (2, 7, 1), (300, 7, 10), (1037, 8, 17),
                                     (515, 14, 32), (700, 7, 4), (129, 20, 9)])
def test_knn_parity(vk, n, dim, k):
    x = rng("gpu-knn", f"{n}-{dim}").uniform(-2.9, 2.9, (n, dim)).astype(np.float32)
    say("knn", n, dim, k)
    idx, d2 = vk.knn(dev(x), k)
    gi, gd = host(idx), host(d2)
    rows, ties = knn_against_exact(x, gi, gd, k)
    say(f"  FP64 reference: {rows} rows, {ties} with a near tie")
    ridx, rd2 = roadmap.knn(x, k)
    np.testing.assert_array_equal(gi, ridx)                 # fixed-order FP32: bit for bit
    np.testing.assert_array_equal(gd, rd2)


def test_knn_ties_and_non_finite(vk):
    x = np.array([[0.5, 0.5], [1, 1], [0, 0], [1, 0], [0, 1], [np.nan, 0], [0.5, 0.5]], np.float32)
    idx, d2 = vk.knn(dev(x), 6)
    gi, gd = host(idx), host(d2)
    rows, ties = knn_against_exact(x, gi, gd, 6)
    say(f"ties and non-finite: {rows} rows, {ties} with a near tie")
    assert ties > 0                                         # the square corners are exact ties
    ridx, rd2 = roadmap.knn(x, 6)
    np.testing.assert_array_equal(gi, ridx)
    np.testing.assert_array_equal(gd, rd2)


def test_knn_full_size_sampled(vk):
    """8,192 roadmap samples of the 7-DoF robot, k = 10 (the benchmark's roadmap); the reference
    recomputes 256 seeded rows."""
    w = workload("prm7_shelf")
    x = w["nodes"]
    idx, d2 = vk.knn(dev(x), w["k"])
    rows = np.sort(np.random.default_rng(2).choice(len(x), 256, replace=False))
    gi, gd = host(idx), host(d2)
    n_rows, ties = knn_against_exact(x, gi[rows], gd[rows], w["k"], rows=rows)
    say(f"full-size kNN, FP64 reference: {n_rows} sampled rows, {ties} with a near tie")
    ridx, rd2 = roadmap.knn(x, w["k"], rows=rows)
    np.testing.assert_array_equal(gi[rows], ridx)
    np.testing.assert_array_equal(gd[rows], rd2)


def test_knn_pairs_parity(vk):
    x = rng("gpu-knn", "pairs").uniform(-1, 1, (900, 7)).astype(np.float32)
    idx, _ = vk.knn(dev(x), 8)
    pairs = host(vk.knn_pairs(idx))
    np.testing.assert_array_equal(pairs, roadmap.knn_pairs(host(idx)))
    # hand-made lists with out-of-range, self and negative entries
    bad = np.array([[1, 7], [0, -1], [2, 0]], np.int32)
    np.testing.assert_array_equal(host(vk.knn_pairs(dev(bad))), roadmap.knn_pairs(bad))


def test_roadmap_edges_parity(vk, orc):
    """kNN roadmap -> pair list -> one persistent launch over the index pairs, against the FP64
    oracle on the materialised endpoints; holes must read 0."""
    w = workload("prm7_shelf", n=600)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    nodes = dev(w["nodes"])
    idx, _ = vk.knn(nodes, 6)
    pairs = vk.knn_pairs(idx)
    flags = host(vk.validate_edges_indexed(r, e, nodes, pairs, resolution=RES))
    p = host(pairs)
    real = p[:, 0] >= 0
    say("roadmap edges", int(real.sum()), "of", len(p), "slots")
    assert np.all(flags[~real] == 0)
    _, cls, _ = orc.edges(w["robot"], w["env"], w["nodes"][p[real, 0]], w["nodes"][p[real, 1]], res=RES)
    bad, near = edge_mismatches(flags[real], cls)
    say(f"  mismatches outside band {bad}, near-contact {near}, collision rate {flags[real].mean():.3f}")
    assert bad == 0


def test_shortcut_edges_parity(vk, orc):
    w = workload("shortcut7_shelf", n=300)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    flags = host(vk.validate_edges_indexed(r, e, dev(w["nodes"]), dev(w["pairs"]), resolution=RES))
    p = w["pairs"]
    _, cls, _ = orc.edges(w["robot"], w["env"], w["nodes"][p[:, 0]], w["nodes"][p[:, 1]], res=RES)
    bad, near = edge_mismatches(flags, cls)
    say(f"shortcut edges {len(p)}: mismatches outside band {bad}, near-contact {near}, "
        f"collision rate {flags.mean():.3f}")
    assert bad == 0


def test_indexed_edges_equal_direct(vk):
    """Index pairs and materialised endpoints give bitwise equal flags; holes are 0 and
    indices past the node array are 1; an empty batch is a no-op."""
    import torch
    w = workload("shortcut7_shelf", n=64)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    nodes, p = w["nodes"], w["pairs"].copy()
    direct = host(vk.validate_edges(r, e, dev(nodes[p[:, 0]]), dev(nodes[p[:, 1]]), resolution=RES))
    p[5] = (-1, -1)
    p[9] = (3, -4)
    p[11] = (len(nodes), 0)
    p[12] = (0, len(nodes) + 100)
    flags = host(vk.validate_edges_indexed(r, e, dev(nodes), dev(p), resolution=RES))
    keep = np.ones(len(p), bool)
    keep[[5, 9, 11, 12]] = False
    np.testing.assert_array_equal(flags[keep], direct[keep])
    assert flags[5] == 0 and flags[9] == 0 and flags[11] == 1 and flags[12] == 1
    empty = vk.validate_edges_indexed(r, e, dev(nodes), torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert empty.numel() == 0
