"""The autotuner's host side (CPU only): its JSON cache round-trips, tolerates a missing or
corrupt file, and workload classes bucket sizes by powers of two."""
import json
import os

from paper_2309_14545_amd import autotune


def test_bucket_is_the_next_power_of_two():
    assert [autotune._bucket(x) for x in (1, 2, 3, 42, 64, 65, 65536, 65537)] == \
        [1, 2, 4, 64, 64, 128, 65536, 131072]


def test_cache_round_trip_and_damage(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune._load(path) == {}                       # missing file
    data = {"dev|dof7|s64|p256|e65536": {"block": 1024, "per_cu": 2, "ms": 0.61}}
    autotune._save(path, data)
    assert autotune._load(path) == data
    assert not [f for f in os.listdir(os.path.dirname(path)) if ".tmp" in f]
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune._load(path) == {}                       # corrupt file: tune again
    autotune._save(path, data)
    assert json.load(open(path)) == data
