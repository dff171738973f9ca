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


def test_tune_set_block_keeps_trajectories_bitwise():
    """Changing the workgroup size between calls (graphs recaptured) leaves forces and
    trajectories bit-identical; layout knobs are refused."""
    import numpy as np
    from paper_2609_07842_amd import vbc
    from paper_2609_07842_amd import workloads as W
    wl = W.fluid(8_000, 0.4, 3.0, seed=5)
    out = []
    for switch in (False, True):
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32", block=256)
        s.set_state(wl.x, wl.v)
        s.step(40, integrator="langevin", seed=3)
        if switch:
            s.tune_set(block=512)
            assert s.options()["block"] == 512
        s.step(40, integrator="langevin", seed=3)
        s.check()
        x, v = s.get_state()
        F, _, _ = s.force(energies=False)
        out.append((x.cpu().numpy(), v.cpu().numpy(), F.cpu().numpy()))
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    o = vbc.Options()
    o.precision = vbc.FP32_MIXED
    o.brick = 2
    st = vbc.lib().vbc_tune_set(s.h, o)
    assert st == vbc.VBC_ERR_UNIMPLEMENTED
