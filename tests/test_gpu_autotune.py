"""The native autotuner (vk_autotune_edges / vk_autotune_states) and its JSON cache: a tuned
setting is a candidate and lands in the file; a class already in the file is applied as it
stands; a damaged file is tuned again and rewritten; flags never depend on the setting."""
import json

import numpy as np
import pytest

from helpers import dev, host, say
from synthetic import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vk():
    import torch
    assert torch.cuda.is_available()
    import paper_2309_14545_amd as vk
    vk.lib()
    return vk


def test_edges_tuning_and_cache(vk, tmp_path):
    from paper_2309_14545_amd import autotune
    w = workload("edges7_shelf", n=4096)
    env = vk.Env(w["env"])
    qa, qb = dev(w["qa"]), dev(w["qb"])
    path = str(tmp_path / "tune.json")
    r = vk.Robot(w["robot"])
    ref = host(vk.validate_edges(r, env, qa, qb))
    block, per_cu, tickets = autotune.tune_edges(r, env, qa, qb, cache=path)
    say("tuned edge launch", block, per_cu, tickets)
    assert block in (64, 128, 256, 512, 1024) and per_cu in (1, 2, 4, 8) and tickets in (4, 8, 16)
    assert block * per_cu <= 2048
    data = json.load(open(path))
    (key, entry), = data.items()
    assert key.startswith("edges|") and "|dof7|" in key and key.endswith("|n4096")
    assert (entry["block"], entry["per_cu"], entry["tickets"]) == (block, per_cu, tickets)
    assert entry["ms"] > 0
    np.testing.assert_array_equal(host(vk.validate_edges(r, env, qa, qb)), ref)
    # a cached class is applied as it stands (192 threads is no candidate, so nothing was timed)
    data[key] = {"block": 192, "per_cu": 3, "tickets": 5, "ms": 1.0}
    json.dump(data, open(path, "w"))
    r2 = vk.Robot(w["robot"])
    assert autotune.tune_edges(r2, env, qa, qb, cache=path) == (192, 3, 5)
    np.testing.assert_array_equal(host(vk.validate_edges(r2, env, qa, qb)), ref)
    # force times it again and replaces the entry
    assert autotune.tune_edges(r2, env, qa, qb, cache=path, force=True)[0] != 192
    assert json.load(open(path))[key]["block"] != 192
    # a damaged file: tuned again, rewritten as valid JSON
    open(path, "w").write("{not json")
    r3 = vk.Robot(w["robot"])
    assert autotune.tune_edges(r3, env, qa, qb, cache=path)[0] in (64, 128, 256, 512, 1024)
    assert list(json.load(open(path))) == [key]


def test_states_tuning_and_cache(vk, tmp_path):
    from paper_2309_14545_amd import autotune
    w = workload("states7", n=20000)
    r, env = vk.Robot(w["robot"]), vk.Env(w["env"])
    q = dev(w["q"])
    ref = host(vk.validate_states(r, env, q))
    path = str(tmp_path / "tune.json")
    # an edge entry already in the file stays as it is
    json.dump({"edges|x": {"block": 64, "per_cu": 1, "tickets": 8, "ms": 2.0}}, open(path, "w"))
    split = autotune.tune_states(r, env, q, cache=path)
    say("tuned states split", split)
    assert split in ((0, 1), (1, 3), (1, 2), (2, 3))
    data = json.load(open(path))
    assert data["edges|x"] == {"block": 64, "per_cu": 1, "tickets": 8, "ms": 2.0}
    key = [k for k in data if k.startswith("states|")][0]
    assert (data[key]["num"], data[key]["den"]) == split
    np.testing.assert_array_equal(host(vk.validate_states(r, env, q)), ref)
    data[key] = {"num": 3, "den": 7, "ms": 1.0}
    json.dump(data, open(path, "w"))
    r2 = vk.Robot(w["robot"])
    assert autotune.tune_states(r2, env, q, cache=path) == (3, 7)
    np.testing.assert_array_equal(host(vk.validate_states(r2, env, q)), ref)
