"""The tuning cache on the CPU (host-only calls of the C ABI): keys name the
architecture, feature set, bin counts and the size classes of scan B and the
grid; tunings round-trip through the JSON file; bad keys and files are
refused."""
import json

import pytest

from paper_1709_06948_amd import mi


def test_key_names_the_workload_classes():
    k = mi.tuning_cache_key("gfx950:sramecc+:xnack-", 3, 32, 32, 277_654, 640 * 640 * 40)
    assert k == "gfx950/f3/b32x32/n19/v24"
    # same size class, same key; the next power of two is another class
    assert mi.tuning_cache_key("gfx950", 3, 32, 32, 262_145, 16_000_000) == k
    assert mi.tuning_cache_key("gfx950", 3, 32, 32, 524_289, 16_000_000).endswith("/n20/v24")
    assert mi.tuning_cache_key("gfx950", 1, 16, 0, 1, 1) == "gfx950/f1/b16x0/n0/v0"


def test_round_trip_and_replace(tmp_path):
    path = str(tmp_path / "tuning.json")
    key = mi.tuning_cache_key("gfx950", 3, 32, 32, 100_000, 2_000_000)
    assert mi.tuning_cache_get(path, key) is None  # no file: an empty cache
    t1 = dict(waves=16, hash_bytes=0, hist_copies=1, stripe_rows=16, wgs_per_cu=2)
    t2 = dict(waves=8, hash_bytes=61440, hist_copies=2, stripe_rows=8, wgs_per_cu=0)
    mi.tuning_cache_put(path, key, t1)
    other = mi.tuning_cache_key("gfx950", 1, 16, 0, 20_000, 40_960)
    mi.tuning_cache_put(path, other, t2)
    assert mi.tuning_cache_get(path, key) == t1
    assert mi.tuning_cache_get(path, other) == t2
    mi.tuning_cache_put(path, key, t2)
    assert mi.tuning_cache_get(path, key) == t2
    # the file is plain JSON: one member per key
    doc = json.load(open(path))
    assert doc == {key: list(t2.values()), other: list(t2.values())}


def test_bad_keys_and_files_are_refused(tmp_path):
    path = str(tmp_path / "tuning.json")
    t = dict(waves=16, hash_bytes=0, hist_copies=1, stripe_rows=16, wgs_per_cu=2)
    for bad in ('gfx"950/f1', "gfx\\950", ""):
        with pytest.raises(mi.MIError):
            mi.tuning_cache_put(path, bad, t)
    with pytest.raises(mi.MIError):
        mi.tuning_cache_key('gfx"950', 1, 16, 0, 1, 1)
    with open(path, "w") as f:
        f.write("not a cache")
    with pytest.raises(mi.MIError):
        mi.tuning_cache_get(path, "gfx950/f1/b16x0/n0/v0")
