"""GPU observables of valency control (neighbours within r_a, core penetrations within r_r)
against the oracle, bit for bit: integer counts decided in FP64 the same way on both sides."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_observables_bit_exact_along_a_trajectory(precision):
    vbc = _vbc()
    wl = W.fluid(3000, 0.5, 4.0, E_a=5.0, seed=12)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision=precision)
    s.set_state(wl.x, wl.v)
    for k in range(3):
        if k:
            s.step(40, integrator="langevin", seed=2)
        z, p, sums = s.observables()
        s.check()
        x = s.get_state()[0].cpu().numpy()
        zr, pr = oracle.observables(x, wl.L, wl.params)
        z, p, sums = z.cpu().numpy(), p.cpu().numpy(), sums.cpu().numpy()
        print(f"[observables] {precision} step {40 * k}: <z> {z.mean():.3f}  pen {p.mean():.3f}", flush=True)
        assert np.array_equal(z, zr) and np.array_equal(p, pr)
        assert sums[0, 0] == zr.sum() and sums[0, 2] == pr.sum()
        assert sums[0, 1] == int((zr > 4.0).sum())


def test_observables_multitype_and_pool_sums():
    vbc = _vbc()
    rng = np.random.default_rng(4)
    N = 2000
    L = W.box_length(N, 0.4)
    types = rng.integers(0, 2, size=N).astype(np.int32)
    pa = W.vbc_params(f=2.0)
    pb = dict(W.vbc_params(f=3.0), r_r=0.8, r_a=1.3, r_l=1.3, r_h=1.7)
    pab = dict(W.vbc_params(f=1.0), r_r=0.9, r_a=1.4, r_l=1.4, r_h=1.8)
    params = [pa, pab, pab, pb]
    x = W.uniform_positions(N, L, 5)
    s = vbc.System(vbc.replica(N, L, params), precision="fp32")
    s.set_state(x, types=types)
    z, p, _ = s.observables()
    zr, pr = oracle.observables(x, L, params, types)
    assert np.array_equal(z.cpu().numpy(), zr) and np.array_equal(p.cpu().numpy(), pr)
    # two replicas in a pool: per-slot sums
    a = W.fluid(1500, 0.3, 2.0, seed=1)
    b = W.fluid(2500, 0.5, 5.0, seed=2)
    auto = [vbc.footprint(vbc.replica(w.N, w.L, w.params), "fp32") for w in (a, b)]
    k_max, stage_cap = max(f["k_max"] for f in auto), max(f["stage_cap"] for f in auto)
    fps = [vbc.footprint(vbc.replica(w.N, w.L, w.params), "fp32", k_max=k_max, stage_cap=stage_cap)
           for w in (a, b)]
    caps = dict(max_replicas=3, max_types=1, max_particles=8000, max_slots=2 * sum(f["slots"] for f in fps),
                max_bricks=2 * sum(f["bricks"] for f in fps), max_cells=2 * sum(f["cells"] for f in fps),
                max_bcap=max(f["bcap"] for f in fps), chains=False)
    pool = vbc.Pool(caps, precision="fp32", k_max=k_max, stage_cap=stage_cap)
    ra = pool.admit(vbc.replica(a.N, a.L, a.params), a.x)
    rb = pool.admit(vbc.replica(b.N, b.L, b.params), b.x)
    z, p, sums = pool.observables()
    sums = sums.cpu().numpy()
    for r, w in ((ra, a), (rb, b)):
        n, off = pool.info(r)
        zr, pr = oracle.observables(w.x, w.L, w.params)
        assert np.array_equal(z.cpu().numpy()[off:off + n], zr)
        assert sums[r, 0] == zr.sum() and sums[r, 2] == pr.sum()
        assert sums[r, 1] == int((zr > w.params["f"]).sum())
    assert (sums[2] == 0).all()
