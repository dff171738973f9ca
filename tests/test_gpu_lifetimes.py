"""GPU bond-lifetime tracker (Section 4) against the oracle's, bit for bit: the same bonds
(decided in FP64 the same way) sampled at the same steps give the same lifetime histogram
and event counts."""
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
def test_bond_tracker_bit_exact_along_a_trajectory(precision):
    vbc = _vbc()
    wl = W.fluid(2000, 0.05, 2.0, E_a=6.0, seed=9)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision=precision, rho_max=1.0)
    s.set_state(wl.x, wl.v)
    tr = s.bond_tracker(max_partners=32, hist_len=64, bin_steps=20)
    ref = oracle.BondTracker(64, 20)
    ref.reset(oracle.bond_pairs(s.get_state()[0].cpu().numpy(), wl.L, wl.params["r_a"]))
    step = 0
    for k in range(40):
        s.step(20, integrator="langevin", seed=4)
        step += 20
        tr.sample()
        ref.sample(oracle.bond_pairs(s.get_state()[0].cpu().numpy(), wl.L, wl.params["r_a"]), step)
        if k % 10 == 9:
            assert tr.stats.cpu().numpy()[0].tolist() == ref.stats.tolist()
    s.check()
    st = tr.stats.cpu().numpy()[0]
    print(f"[lifetimes] {precision}: formed {st[0]}, broken {st[1]} (+{st[2]} censored), "
          f"median {tr.median_lifetime()} steps", flush=True)
    assert np.array_equal(tr.hist.cpu().numpy()[0], ref.hist)
    assert st.tolist() == ref.stats.tolist() and st[3] == 0 and st[1] > 50


def test_bond_tracker_in_a_pool_and_capacity():
    vbc = _vbc()
    a = W.fluid(1500, 0.05, 1.0, E_a=6.0, seed=1)
    b = W.fluid(2500, 0.05, 3.0, E_a=6.0, seed=2)
    auto = [vbc.footprint(vbc.replica(w.N, w.L, w.params), "fp32", rho_max=1.0) for w in (a, b)]
    k_max, stage_cap = max(f["k_max"] for f in auto), max(f["stage_cap"] for f in auto)
    fps = [vbc.footprint(vbc.replica(w.N, w.L, w.params), "fp32", k_max=k_max, stage_cap=stage_cap,
                         rho_max=1.0) for w in (a, b)]
    caps = dict(max_replicas=3, max_types=1, max_particles=8000, max_slots=2 * sum(f["slots"] for f in fps),
                max_bricks=2 * sum(f["bricks"] for f in fps), max_cells=2 * sum(f["cells"] for f in fps),
                max_bcap=max(f["bcap"] for f in fps), chains=False)
    pool = vbc.Pool(caps, precision="fp32", k_max=k_max, stage_cap=stage_cap, rho_max=1.0)
    ra = pool.admit(vbc.replica(a.N, a.L, a.params), a.x, a.v)
    rb = pool.admit(vbc.replica(b.N, b.L, b.params), b.x, b.v)
    tr = pool.bond_tracker(max_partners=16, hist_len=32, bin_steps=10)
    refs = {}
    x = pool.get_state()[0].cpu().numpy()
    for r, w in ((ra, a), (rb, b)):
        n, off = pool.info(r)
        refs[r] = oracle.BondTracker(32, 10)
        refs[r].reset(oracle.bond_pairs(x[off:off + n], w.L, w.params["r_a"]))
    for k in range(1, 21):
        pool.step(10, integrator="langevin", seed=5)
        tr.sample()
        x = pool.get_state()[0].cpu().numpy()
        for r, w in ((ra, a), (rb, b)):
            n, off = pool.info(r)
            refs[r].sample(oracle.bond_pairs(x[off:off + n], w.L, w.params["r_a"]), 10 * k)
    pool.check()
    hist, stats = tr.hist.cpu().numpy(), tr.stats.cpu().numpy()
    for r in (ra, rb):
        assert np.array_equal(hist[r], refs[r].hist) and stats[r].tolist() == refs[r].stats.tolist()
    assert (hist[3 - ra - rb] == 0).all() and (stats[3 - ra - rb] == 0).all()
    # one partner at most: particles with two bonds overflow and say so
    small = pool.bond_tracker(max_partners=1, hist_len=4, bin_steps=10)
    pool.step(10, integrator="langevin", seed=5)
    small.sample()
    assert small.stats.cpu().numpy()[rb, 3] > 0


def test_lifetime_sweep_exchange_geometry_repartners_faster():
    """Section 4, Fig. 7: bond lifetimes grow with saturation for the standard geometry,
    while VBC(1.29, 1.50, 0.30) keeps them short under strong binding."""
    from paper_2609_07842_amd import lifetimes
    res = lifetimes.lifetime_sweep(fs=(1,), beta_Ea=(1.0, 8.0), N=2000, equil=4000, steps=8000,
                                   every=10)["results"]
    for k, v in res.items():
        print(f"[lifetimes] {k}: p {v['saturation']:.3f} tau_rate {v['tau_rate']:.1f} "
              f"tau_median {v['tau_median']}", flush=True)
        assert v["overflow"] == 0
    std_w, std_s = res["standard f=1 betaEa=1"], res["standard f=1 betaEa=8"]
    tun_s = res["exchange f=1 betaEa=8"]
    assert std_s["saturation"] > std_w["saturation"] and std_s["tau_rate"] > 5 * std_w["tau_rate"]
    assert tun_s["tau_rate"] < std_s["tau_rate"] / 5
