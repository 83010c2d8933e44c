"""GPU parity of validate_edges (persistent batched launch) and validate_edges_per_edge
against the FP64 oracle, plus schedule invariance and degenerate edges."""
import numpy as np
import pytest

from helpers import dev, host, say, edge_mismatches, state_mismatches
from synthetic import workload, rng, uniform_edges

pytestmark = pytest.mark.gpu
RES = 1.0 / 32.0


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    yield vk


@pytest.mark.parametrize("name", ["edges7_shelf", "edges8_shelf", "edges8p_shelf"])
@pytest.mark.parametrize("per_edge", [False, True], ids=["batched", "per_edge"])
def test_edges_parity(vk, orc, name, per_edge):
    w = workload(name, n=1500)
    say("validate_edges", name, "per_edge" if per_edge else "batched", "E", len(w["qa"]))
    flags = host(vk.validate_edges(vk.Robot(w["robot"]), vk.Env(w["env"]), dev(w["qa"]),
                                   dev(w["qb"]), resolution=RES, per_edge=per_edge))
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"], w["qb"], res=RES)
    bad, near = edge_mismatches(flags, cls)
    say(f"  mismatches outside band {bad}, near-contact {near}, collision rate {flags.mean():.3f}")
    assert bad == 0


@pytest.mark.parametrize("name", ["edges7_shelf", "edges8_shelf", "edges8p_shelf"])
def test_self_only_edges_parity(vk, orc, name):
    """No obstacles: every colliding edge collides with the robot itself, so the self-block
    gates (bounding spheres, then bounding capsules, one of them kept per lane in half
    precision) decide alone whether a pair is tested."""
    w = workload(name, n=1500)
    flags = host(vk.validate_edges(vk.Robot(w["robot"]), vk.Env({}), dev(w["qa"]), dev(w["qb"]),
                                   resolution=RES))
    _, cls, _ = orc.edges(w["robot"], {}, w["qa"], w["qb"], res=RES)
    bad, near = edge_mismatches(flags, cls)
    say(f"self-only edges {name}: mismatches {bad}, near-contact {near}, rate {flags.mean():.3f}")
    assert bad == 0 and flags.any()


@pytest.mark.parametrize("name", ["edges7_shelf", "edges8_shelf"])
def test_edges_full_size_sampled(vk, orc, name):
    """The full 65,536-edge shelf batches (7-DoF, the benchmark's; 8-DoF, 60 spheres and 400
    pairs) in the default launch; the oracle checks a seeded sample of 600 edges."""
    w = workload(name)
    E = len(w["qa"])
    say("validate_edges full size", E)
    flags = host(vk.validate_edges(vk.Robot(w["robot"]), vk.Env(w["env"]), dev(w["qa"]),
                                   dev(w["qb"]), resolution=RES))
    idx = np.sort(np.random.default_rng(11).choice(E, 600, replace=False))
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"][idx], w["qb"][idx], res=RES)
    assert edge_mismatches(flags[idx], cls)[0] == 0


def test_schedule_invariance(vk):
    """Flags do not depend on the launch shape or on batching: bitwise equal across workgroup
    sizes, workgroups per CU and the one-launch-per-edge path."""
    w = workload("edges8_shelf", n=3000)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    ref = host(vk.validate_edges(r, e, qa, qb, per_edge=True))
    for block, bpc, tickets in ((64, 1, 8), (128, 3, 1), (256, 8, 16), (192, 2, 4), (256, 1, 64),
                                (512, 4, 8), (1024, 2, 8), (960, 1, 3)):
        say("launch", block, bpc, tickets)
        r.set_edge_launch(block, bpc, tickets)
        np.testing.assert_array_equal(host(vk.validate_edges(r, e, qa, qb)), ref)


def test_small_batch_launch_shapes(vk):
    """Batches too small to give every CU a workgroup of the tuned size run in smaller
    workgroups over more CUs: the flags of every prefix batch, at sizes around those thresholds,
    equal the full batch's."""
    w = workload("edges7_shelf", n=8192)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = w["qa"], w["qb"]
    for block, bpc in ((1024, 2), (256, 8)):
        r.set_edge_launch(block, bpc, 8)
        full = host(vk.validate_edges(r, e, dev(qa), dev(qb)))
        assert 0 < full.mean() < 1
        for E in (1, 2, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097):
            say("launch", block, bpc, "edges", E)
            got = host(vk.validate_edges(r, e, dev(qa[:E]), dev(qb[:E])))
            np.testing.assert_array_equal(got, full[:E])


def test_explicit_state_counts(vk, orc):
    import torch
    w = workload("edges7_shelf", n=800)
    g = np.random.default_rng(2)
    ns = g.integers(2, 300, len(w["qa"])).astype(np.int32)
    flags = host(vk.validate_edges(vk.Robot(w["robot"]), vk.Env(w["env"]), dev(w["qa"]),
                                   dev(w["qb"]), n_states=dev(ns)))
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"], w["qb"], n_states=ns)
    assert edge_mismatches(flags, cls)[0] == 0


def test_endpoints_only_equals_states(vk):
    """With two states per edge the edge flag is exactly the OR of the two endpoint states'
    flags from validate_states (both paths evaluate the very same FP32 configurations)."""
    w = workload("edges7_shelf", n=2000)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    ns = np.full(len(w["qa"]), 2, np.int32)
    fe = host(vk.validate_edges(r, e, dev(w["qa"]), dev(w["qb"]), n_states=dev(ns)))
    fa = host(vk.validate_states(r, e, dev(np.ascontiguousarray(w["qa"].T))))
    fb = host(vk.validate_states(r, e, dev(np.ascontiguousarray(w["qb"].T))))
    np.testing.assert_array_equal(fe, fa | fb)


def test_fine_resolution_long_edges(vk, orc):
    """Resolution 1/256 rad: up to ~1,500 states per edge, ~24 rake steps."""
    w = workload("edges7_shelf", n=120)
    flags = host(vk.validate_edges(vk.Robot(w["robot"]), vk.Env(w["env"]), dev(w["qa"]),
                                   dev(w["qb"]), resolution=1.0 / 256.0))
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"], w["qb"], res=1.0 / 256.0)
    assert edge_mismatches(flags, cls)[0] == 0


def test_degenerate_edges(vk, orc):
    import torch
    w = workload("edges7_shelf", n=256)
    qa, qb = w["qa"].copy(), w["qb"].copy()
    qb[:40] = qa[:40]                       # zero length: two copies of one state
    qa[40, 2] = np.nan                      # non-finite endpoint -> colliding
    qb[41, 0] = np.inf
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    flags = host(vk.validate_edges(r, e, dev(qa), dev(qb)))
    assert flags[40] == 1 and flags[41] == 1
    _, cls, _ = orc.edges(w["robot"], w["env"], qa, qb)
    assert edge_mismatches(flags, cls)[0] == 0
    # zero-length edges agree with their single state
    cm, _ = orc.states(w["robot"], w["env"], qa[:40].T)
    assert state_mismatches(flags[:40], cm)[0] == 0
    # empty batch is a no-op
    out = vk.validate_edges(r, e, torch.zeros((0, 7), device="cuda"), torch.zeros((0, 7), device="cuda"))
    assert out.numel() == 0


def test_argument_errors(vk):
    import torch
    w = workload("edges7_shelf", n=4)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa = dev(w["qa"])
    with pytest.raises(vk.VkError):
        vk.validate_edges(r, e, qa, qa, resolution=0.0)
    with pytest.raises(vk.VkError):
        vk.validate_edges(r, e, qa, qa, resolution=float("nan"))
    with pytest.raises(ValueError):
        vk.validate_edges(r, e, qa, qa[:, :6].contiguous())


def test_edges_beyond_the_state_limit(vk):
    """An edge of more than 2^24 states is not validated and reads 1: endpoints far apart (the
    computed count saturates at 2^31 - 1) and an explicit count of 2^24 + 1.  Shorter edges in
    the same launch keep their flags."""
    w = workload("edges7_shelf", n=64)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    base = host(vk.validate_edges(r, e, dev(w["qa"]), dev(w["qb"])))
    qa, qb = w["qa"].copy(), w["qb"].copy()
    qb[3, 1] = np.float32(1e9)                        # 3.2e10 states at 1/32: saturated
    qa[4], qb[4] = 0.0, 0.0
    qb[4, 0] = np.float32(2.0 ** 19)                  # 2^24 + 1 states at 1/32
    assert vk.edge_states(qa[3], qb[3]) == 2 ** 31 - 1
    assert vk.edge_states(qa[4], qb[4]) == 2 ** 24 + 1
    flags = host(vk.validate_edges(r, e, dev(qa), dev(qb)))
    assert flags[3] == 1 and flags[4] == 1
    keep = np.ones(len(qa), bool)
    keep[[3, 4]] = False
    np.testing.assert_array_equal(flags[keep], base[keep])
    ns = np.full(len(qa), 5, np.int32)
    ns[7] = 2 ** 24 + 1
    f2 = host(vk.validate_edges(r, e, dev(w["qa"]), dev(w["qb"]), n_states=dev(ns)))
    assert f2[7] == 1


@pytest.mark.parametrize("res", [1.0 / 256.0, 1.0 / 1024.0])
def test_long_edges_split_over_waves(vk, orc, res):
    """Long edges (fine resolutions: up to ~1,500 and ~6,000 states) with their rake split over
    several waves give bitwise the flags of one wave per edge, for every part count, and agree
    with the oracle outside the band."""
    w = workload("edges7_shelf", n=1200 if res > 1e-3 else 300)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    ref = host(vk.validate_edges(r, e, qa, qb, resolution=res))
    for parts in (2, 3, 4, 8, 64):
        r.set_edge_parts(parts)
        assert r.edge_parts == parts
        np.testing.assert_array_equal(host(vk.validate_edges(r, e, qa, qb, resolution=res)), ref,
                                      err_msg=f"parts {parts}")
    idx = np.sort(np.random.default_rng(6).choice(len(w["qa"]), 60, replace=False))
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"][idx], w["qb"][idx], res=res)
    bad, near = edge_mismatches(ref[idx], cls)
    say(f"long edges at {res:.5f} rad: {len(ref)} edges, rate {ref.mean():.3f}, sample mismatches "
        f"{bad}, near {near}")
    assert bad == 0


def test_parts_with_explicit_counts_and_indexed_edges(vk):
    """Parts with explicit state counts (2 .. 5,000) and with index-pair edges (holes and
    out-of-range indices included) equal one wave per edge."""
    import torch
    w = workload("edges7_shelf", n=900)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    ns = torch.from_numpy(np.random.default_rng(9).integers(2, 5000, 900).astype(np.int32)).cuda()
    nodes = torch.cat([qa, qb])
    pairs = torch.stack([torch.arange(900, dtype=torch.int32), 900 + torch.arange(900, dtype=torch.int32)], 1)
    pairs[5] = torch.tensor([-1, -1], dtype=torch.int32)
    pairs[7] = torch.tensor([3, 5000], dtype=torch.int32)
    pairs = pairs.cuda()
    ref_n = host(vk.validate_edges(r, e, qa, qb, n_states=ns))
    ref_i = host(vk.validate_edges_indexed(r, e, nodes, pairs))
    assert ref_i[5] == 0 and ref_i[7] == 1
    for parts in (2, 5, 16):
        r.set_edge_parts(parts)
        np.testing.assert_array_equal(host(vk.validate_edges(r, e, qa, qb, n_states=ns)), ref_n)
        np.testing.assert_array_equal(host(vk.validate_edges_indexed(r, e, nodes, pairs)), ref_i)


@pytest.mark.parametrize("name", ["edges7_shelf", "edges8_shelf", "edges8p_shelf"])
def test_small_batches_split_over_test_ranges(vk, orc, name):
    """Small edge batches with each edge's walk split over ranges of its tests (environment
    parts and self blocks, each range posing the earlier steps over the edge's whole rake) give
    bitwise the flags of the unsplit walk, for range counts from two to one per test, at ragged
    sizes, with rake parts, with explicit state counts and with index-pair edges; the automatic
    choice agrees with the oracle outside the band."""
    import torch
    w = workload(name, n=700)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    ns = torch.from_numpy(np.random.default_rng(11).integers(2, 400, 700).astype(np.int32)).cuda()
    nodes = torch.cat([qa, qb])
    pairs = torch.stack([torch.arange(700, dtype=torch.int32),
                         700 + torch.arange(700, dtype=torch.int32)], 1)
    pairs[3] = torch.tensor([-1, 2], dtype=torch.int32)
    pairs = pairs.cuda()
    r.set_edge_ranges(0)
    assert r.edge_ranges() == 0
    ref = host(vk.validate_edges(r, e, qa, qb)).copy()
    ref_n = host(vk.validate_edges(r, e, qa, qb, n_states=ns)).copy()
    ref_i = host(vk.validate_edges_indexed(r, e, nodes, pairs)).copy()
    assert 0 < ref.mean() < 1 and ref_i[3] == 0
    for k in (2, 3, 7, 16, 32):
        r.set_edge_ranges(k)
        for E in (1, 63, 65, 700):
            got = host(vk.validate_edges(r, e, qa[:E].contiguous(), qb[:E].contiguous()))
            np.testing.assert_array_equal(got, ref[:E], err_msg=f"{name} ranges {k} E {E}")
        np.testing.assert_array_equal(host(vk.validate_edges(r, e, qa, qb, n_states=ns)), ref_n)
        np.testing.assert_array_equal(host(vk.validate_edges_indexed(r, e, nodes, pairs)), ref_i)
        r.set_edge_parts(2)
        np.testing.assert_array_equal(host(vk.validate_edges(r, e, qa, qb)), ref,
                                      err_msg=f"{name} ranges {k} parts 2")
        r.set_edge_parts(1)
    for bad in (-2, 33):
        with pytest.raises(vk.VkError):
            r.set_edge_ranges(bad)
    r.set_edge_ranges(-1)
    auto = host(vk.validate_edges(r, e, qa, qb))
    np.testing.assert_array_equal(auto, ref)
    idx = np.arange(0, 700, 7)
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"][idx], w["qb"][idx], res=RES)
    bad, near = edge_mismatches(auto[idx], cls)
    say(f"test ranges {name}: {len(auto)} edges, rate {auto.mean():.3f}, sample mismatches {bad}, "
        f"near {near}")
    assert bad == 0


def test_queue_ring_over_many_launches(vk, orc):
    """Edge launches take the slots of the stream's queue ring in turn and the ring is zeroed
    when it wraps: 80 launches in a row (two and a half wraps), without a synchronisation
    between them, interleaved with split launches (which zero a slot of their own), on a second
    stream too, all give the first launch's flags, and those agree with the oracle."""
    import torch
    w = workload("edges7_shelf", n=300)
    r, e = vk.Robot(w["robot"]), vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    r.set_edge_ranges(0)
    ref = host(vk.validate_edges(r, e, qa, qb)).copy()
    _, cls, _ = orc.edges(w["robot"], w["env"], w["qa"], w["qb"], res=1.0 / 32.0)
    assert edge_mismatches(ref, cls)[0] == 0 and 0 < ref.mean() < 1
    r.set_edge_ranges(-1)
    small_ref = ref[:17]
    outs, smalls = [], []
    for i in range(80):
        outs.append(vk.validate_edges(r, e, qa, qb))
        if i % 7 == 3:                        # 17 edges: split over test ranges automatically
            smalls.append(vk.validate_edges(r, e, qa[:17].contiguous(), qb[:17].contiguous()))
    for o in outs:
        np.testing.assert_array_equal(host(o), ref)
    for o in smalls:
        np.testing.assert_array_equal(host(o), small_ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = [vk.validate_edges(r, e, qa, qb) for _ in range(40)]
    side.synchronize()
    for o in got:
        np.testing.assert_array_equal(host(o), ref)
