"""GPU check of valency control on a short sweep: stronger binding raises <z> towards the
valency and lowers the fraction of over-coordinated particles (Section 3, Fig. 2), and more
of the particles end up in loop-carrying clusters (Section 3, cyclisation)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_binding_raises_coordination_towards_valency():
    from paper_2609_07842_amd import valency
    res = valency.saturation_sweep(fs=(1, 3), beta_Ea=(1.0, 8.0), N=4000, rho=0.05, steps=8000,
                                   sample_every=1000)["results"]
    for f in (1, 3):
        weak, strong = res[f"f={f} betaEa=1"], res[f"f={f} betaEa=8"]
        keys = ("z", "P_err", "saturation", "P_inf", "x_cyc")
        print(f"[valency] f={f}: weak {[round(weak[k], 4) for k in keys]}  "
              f"strong {[round(strong[k], 4) for k in keys]}", flush=True)
        assert strong["z"] > weak["z"]
        assert strong["z"] <= f + 0.25
    assert res["f=1 betaEa=8"]["P_err"] < 0.05
    weak, strong = res["f=3 betaEa=1"], res["f=3 betaEa=8"]
    assert strong["x_cyc"] > weak["x_cyc"]
    # a valency-1 fluid holds monomers and dimers, loops only from rare transient triangles
    assert res["f=1 betaEa=8"]["x_cyc"] < 0.03
    import numpy as np
    from paper_2609_07842_amd import workloads as W
    V = W.box_length(4000, 0.05) ** 3
    for r in res.values():
        # the size histograms hold every cluster: their sum is the mean number of clusters
        assert np.sum(r["rho_s_all"]) * V == pytest.approx(r["clusters_per_particle"] * 4000, rel=1e-9)
        assert 0.0 <= r["P_inf"] <= 1.0 and 0.0 <= r["x_cyc"] <= 1.0


def test_counter_geometries_suppress_core_penetration():
    """Section 6.2 (Fig. 12) on a short run (4 x 10^4 steps): at a deep well (E_a = 5) the
    uncorrected soft core collapses with many particles inside each other's core, while the
    standard, partial and blind counting shells keep core penetrations at a fraction of
    that; at a shallow well (E_a = 0.5) nothing collapses.  The standard shell also keeps
    the contacts within r_a below its cap and far below the uncorrected system's."""
    from paper_2609_07842_amd import valency
    res = valency.stability_sweep(E_as=(0.5, 5.0), steps=40_000, sample_every=1000)["results"]
    for g, r in res.items():
        print(f"[stability] {g}: " + ", ".join(f"E_a={e}: z {v['contacts']:.3f} pen {v['penetrations']:.4f}"
                                               for e, v in r.items()), flush=True)
    # thermal excursions into the soft core (V_r(0.9) = 0.7 kT) give about 0.06 penetrations
    # per particle in every geometry at the shallow well; at the deep one the uncorrected
    # core collapses (more than one penetration per particle), the counting shells stay
    # within a few times the thermal level, the partial shell lowest (Fig. 12(b))
    none5 = res["none"]["5"]["penetrations"]
    assert none5 > 1.0
    for g in res:
        assert res[g]["0.5"]["penetrations"] < 0.1
    for g in ("standard", "partial", "blind"):
        assert res[g]["5"]["penetrations"] < none5 / 5
    assert res["partial"]["5"]["penetrations"] < res["standard"]["5"]["penetrations"]
    assert res["standard"]["5"]["penetrations"] < 0.1
    # contacts within r_a: the standard shell saturates below its cap f = 12, the
    # uncorrected system reaches about 20 (Fig. 12(a))
    assert res["standard"]["5"]["contacts"] < 12.0
    assert res["standard"]["5"]["contacts"] < res["none"]["5"]["contacts"] / 2
