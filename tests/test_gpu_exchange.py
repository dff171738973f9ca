"""Energy along the partner-exchange path (Section 4) on the GPU against the oracle: every
point of the path is one replica of a batched handle."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_exchange_path_energies_match_oracle():
    from paper_2609_07842_amd import exchange as E
    geoms = [(1.5, 2.0, 0.0), (1.29, 1.50, 0.30), (1.35, 1.8, 0.1)]
    fs = (1, 3, 5)
    lams = np.linspace(0.0, 1.0, 11)
    U = E.profiles(geoms, fs, points=len(lams))
    for k, (rl, rh, dl) in enumerate(geoms):
        for j, f in enumerate(fs):
            p = W.vbc_params(E_a=2.0, f=float(f), r_l=rl, r_h=rh, delta=dl)
            ref = [oracle.evaluate(E.path_positions(p, f, lam), E.BOX, p)["U"] for lam in lams]
            assert np.allclose(U[k, j], ref, rtol=1e-12, atol=1e-12)


def test_exchange_tuned_geometry_lowers_the_barrier():
    """The standard geometry must break the old bond before the new one forms (barrier =
    E_a, the count sees the newcomer first); VBC(1.29, 1.50, 0.30) lowers it at every
    valency the path covers."""
    from paper_2609_07842_amd import exchange as E
    fs = (1, 2, 3, 4, 5)
    U = E.profiles([(1.5, 2.0, 0.0), (1.29, 1.50, 0.30)], fs, points=41, E_a=2.0)
    std = [E.barrier_and_trap(U[0, j])[0] for j in range(len(fs))]
    tuned = [E.barrier_and_trap(U[1, j])[0] for j in range(len(fs))]
    print(f"[exchange] barriers standard {np.round(std, 3).tolist()} tuned {np.round(tuned, 3).tolist()}", flush=True)
    assert np.allclose(std, 2.0, atol=1e-9)
    assert all(t < s - 0.5 for t, s in zip(tuned, std))
