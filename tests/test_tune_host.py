"""Autotuner cache (host side, no GPU): keys, round trip, lookup of the committed choices."""
import json

from paper_2609_07842_amd import tune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    assert tune.lookup("x", path) is None
    tune.save_cache({"x": {"brick": 3, "block": 256, "steps_per_s": 1.0,
                           "kernel_sha256": tune.kernel_hash()}}, path)
    assert tune.lookup("x", path) == {"brick": 3, "block": 256}
    assert tune.stale("x", path) is None
    with open(path) as fh:
        assert json.load(fh)["x"]["steps_per_s"] == 1.0


def test_entries_timed_with_other_kernels_are_ignored(tmp_path):
    path = str(tmp_path / "t.json")
    tune.save_cache({"x": {"brick": 3, "block": 256, "kernel_sha256": "0" * 64},
                     "y": {"brick": 4, "block": 512}}, path)
    assert tune.lookup("x", path) is None and tune.lookup("y", path) is None
    assert tune.stale("x", path) == "timed with another kernel source"


def test_keys_name_device_and_workload():
    from paper_2609_07842_amd import serve
    k = tune.fluid_key(1_000_000, 0.5, "fp32", device="gfx950x256CU")
    assert k == "gfx950x256CU|fluid|N=1000000|rho=0.5|fp32"
    kp = tune.pool_key(serve.ServerConfig(), device="gfx950x256CU")
    assert kp.startswith("gfx950x256CU|pool|rho=0.3|N=1000-200000|fp32")
    km = tune.melt_key("fp32", device="gfx950x256CU")
    assert km == "gfx950x256CU|melt|N=1000000|rho=0.85|fp32"


def test_committed_choices_are_valid_layouts():
    cache = tune.load_cache()
    for key, e in cache.items():
        assert 1 <= e["brick"] <= 6, key
        assert e["block"] % 64 == 0 and 64 <= e["block"] <= 1024, key
        # the choice is the fastest candidate that was timed
        best = max(e["candidates"], key=lambda c: c.get("steps_per_s", c.get("particle_steps_per_s")))
        assert (best["brick"], best["block"]) == (e["brick"], e["block"]), key
