"""The seeded input generators (CPU only): every parity test and the benchmark rely on them
drawing the same arrays every time, in the canonical FP32 layout, with the sizes and shapes the
workloads are described with."""
import numpy as np
import pytest

from synthetic import pack_edge_sets, workload

NAMES = ["states7", "edges7_shelf", "edges8_shelf", "edges8p_shelf", "states14_cloud", "cost7",
         "prm7_shelf", "shortcut7_shelf", "mixed"]


def _arrays(x, path=""):
    if isinstance(x, dict):
        for k in sorted(x):
            yield from _arrays(x[k], f"{path}/{k}")
    elif isinstance(x, (list, tuple)):
        for i, v in enumerate(x):
            yield from _arrays(v, f"{path}[{i}]")
    elif isinstance(x, np.ndarray):
        yield path, x


@pytest.mark.parametrize("name", NAMES)
def test_workloads_are_reproducible(name):
    a, b = workload(name, n=64), workload(name, n=64)
    pa, pb = list(_arrays(a)), list(_arrays(b))
    assert [p for p, _ in pa] == [p for p, _ in pb] and pa
    for (p, x), (_, y) in zip(pa, pb):
        assert x.dtype == y.dtype and x.shape == y.shape, p
        np.testing.assert_array_equal(x, y, err_msg=p)


def test_mixed_variants_differ():
    """The benchmark times three mixed batches; each variant is its own seeded draw."""
    a, b = workload("mixed", n=16), workload("mixed", n=16, variant=1)
    assert a["sets"] != b["sets"]
    assert not np.array_equal(a["qa"][1][:1], b["qa"][1][:1])


def test_canonical_layouts_and_sizes():
    w = workload("edges7_shelf")
    assert w["qa"].dtype == np.float32 and w["qa"].shape == (65536, 7) == w["qb"].shape
    r = w["robot"]
    assert r["dof"] == 7 and len(r["sphere_link"]) == 42 and len(r["self_pairs"]) == 540
    assert len(w["env"]["boxes"]) == 100 and len(w["env"]["capsules"]) == 50
    w8 = workload("edges8_shelf", n=8)
    assert len(w8["robot"]["sphere_link"]) == 60 and len(w8["robot"]["self_pairs"]) == 400
    s = workload("states7")
    assert s["q"].shape == (7, 4096) and s["q"].dtype == np.float32     # SoA [dof][n]
    c = workload("states14_cloud", n=16)
    assert c["q"].shape == (14, 16) and len(c["env"]["spheres"]) == 20300
    assert len(c["robot"]["sphere_link"]) == 120 and len(c["robot"]["self_pairs"]) == 1500
    t = workload("cost7", n=4)
    assert t["q"].shape == (7, 4 * 64)


def test_mixed_batch_packing():
    w = workload("mixed", n=12)
    qa, qb, sets, total = pack_edge_sets(w)
    assert qa.dtype == np.float32 and qa.shape == qb.shape
    off = out = 0
    for k, (ri, ei, o, ne, oo) in enumerate(sets):
        dof = w["robots"][ri]["dof"]
        assert (o, oo) == (off, out) and ne == len(w["qa"][k])
        np.testing.assert_array_equal(qa[o:o + ne * dof].reshape(ne, dof), w["qa"][k])
        off += ne * dof
        out += ne
    assert total == out and qa.size == off
