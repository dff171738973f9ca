"""Energy landscape of the partner exchange (Section 4) on the GPU against the oracle: every
grid point is one replica of a batched handle."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_exchange_landscape_energies_match_oracle():
    from paper_2609_07842_amd import exchange as E
    geoms = [(1.5, 2.0, 0.0), (1.29, 1.50, 0.30), (1.35, 1.8, 0.1)]
    fs = (1, 3, 5)
    U, radii = E.landscapes(geoms, fs, points=9)
    rng = np.random.default_rng(0)
    for k, (rl, rh, dl) in enumerate(geoms):
        for j, f in enumerate(fs):
            p = W.vbc_params(E_a=2.0, f=float(f), r_l=rl, r_h=rh, delta=dl)
            for a, b in rng.integers(0, 9, size=(8, 2)):
                ref = oracle.evaluate(E.positions(p, f, radii[k][a], radii[k][b]), E.BOX, p)["U"]
                assert U[k, j, a, b] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_exchange_tuned_geometry_lowers_the_barrier():
    """The standard geometry loses the old bond before the new one forms (barrier ~ E_a:
    the count sees the newcomer first); VBC(1.29, 1.50, 0.30) lowers the barrier by an
    order of magnitude at every valency the landscape covers."""
    from paper_2609_07842_amd import exchange as E
    fs = (1, 2, 3, 4, 5)
    U, radii = E.landscapes([(1.5, 2.0, 0.0), (1.29, 1.50, 0.30)], fs, points=31, E_a=2.0)
    std = [E.barrier_and_trap(U[0, j], radii[0]) for j in range(len(fs))]
    tuned = [E.barrier_and_trap(U[1, j], radii[1]) for j in range(len(fs))]
    print(f"[exchange] standard {[(round(b, 3), t) for b, t in std]}", flush=True)
    print(f"[exchange] tuned    {[(round(b, 3), t) for b, t in tuned]}", flush=True)
    assert all(b > 1.8 and not t for b, t in std)
    assert all(bt < bs / 5 for (bt, _), (bs, _) in zip(tuned, std))
    assert not any(t for _, t in tuned)  # and has no trap, as Section 4 states
