"""GPU test of the precision claim on a reduced study: FP64 forces within 1e-10 and FP32
forces within 1e-5 of the oracle (normwise, sampled particles) along Langevin trajectories,
and the trajectory statistics (U/N, mean neighbours within r_a, fraction above the valency)
of the two precisions close to each other."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_fp32_against_fp64_and_oracle_along_trajectories():
    import precision_study as P
    res = P.study(N=20_000, rho=0.3, fs=(2, 5), steps=400, every=200, sample=128, seed=4)
    for f, r in res["results"].items():
        c = r["compare"]
        print(f"[precision] f={f}: {c}", flush=True)
        assert c["max_force_err_fp64"] <= 1e-10
        assert c["max_force_err_fp32"] <= 1e-5
        u64, u32 = c["U_per_N"]
        assert abs(u32 - u64) <= 0.02 * abs(u64)
        z64, z32 = c["z"]
        assert abs(z32 - z64) <= 0.02 * z64
        p64, p32 = c["P_err"]
        assert abs(p32 - p64) <= 0.01
