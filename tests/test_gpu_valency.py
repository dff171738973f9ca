"""GPU check of valency control on a short sweep: stronger binding raises <z> towards the
valency and lowers the fraction of over-coordinated particles (Section 3, Fig. 2)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_binding_raises_coordination_towards_valency():
    from paper_2609_07842_amd import valency
    res = valency.saturation_sweep(fs=(1, 3), beta_Ea=(1.0, 8.0), N=4000, rho=0.05, steps=8000,
                                   sample_every=1000)["results"]
    for f in (1, 3):
        weak, strong = res[f"f={f} betaEa=1"], res[f"f={f} betaEa=8"]
        print(f"[valency] f={f}: weak {weak}  strong {strong}", flush=True)
        assert strong["z"] > weak["z"]
        assert strong["z"] <= f + 0.25
    assert res["f=1 betaEa=8"]["P_err"] < 0.05
