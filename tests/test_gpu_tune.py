"""GPU test of the autotuner: it times candidate layouts on the device, skips those the
device cannot hold, caches the fastest, and the cached layout runs."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_tune_fluid_small(tmp_path):
    from paper_2609_07842_amd import tune, vbc
    from paper_2609_07842_amd import workloads as W
    path = str(tmp_path / "tuned.json")
    best = tune.tune_fluid(N=20_000, rho=0.3, f=2.0, precision="fp32", warmup=40, steps=40,
                           bricks=(3, 4), blocks=(128, 256), path=path, log=print)
    assert best["steps_per_s"] > 0
    got = tune.lookup(tune.fluid_key(20_000, 0.3, "fp32"), path)
    assert got == {"brick": best["brick"], "block": best["block"]}
    wl = W.fluid(20_000, 0.3, 2.0, seed=3)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32", **got)
    s.set_state(wl.x, wl.v)
    s.step(10, integrator="langevin")
    s.check()
    assert s.options()["block"] == got["block"]
