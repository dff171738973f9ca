"""GPU parity of chain exclusions (binding between stickers adjacent along a strand
forbidden, Section 6.1) against the oracle: forces, counts and energies in both
precisions, the neighbour list unchanged, and an FP64 Langevin trajectory with bonds."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _normwise(a, b):
    return np.linalg.norm(np.asarray(a) - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300)


def _melt():
    return W.polymer_melt(nchains=40, nbeads=50, seed=7)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_exclusion_parity(precision, tol):
    from paper_2609_07842_amd import vbc
    wl = _melt()
    span = 5  # stickers every fifth bead: neighbouring stickers of a chain are excluded
    ref = oracle.evaluate(wl.x, wl.L, wl.params, wl.types, wl.mask, chain_len=50, excl_span=span)
    ref0 = oracle.evaluate(wl.x, wl.L, wl.params, wl.types, wl.mask)
    assert np.abs(ref["n"] - ref0["n"]).max() > 0.5  # exclusions matter here
    Ub, Fb = oracle.bonds_energy_forces(wl.x, wl.L, wl.bonds, wl.k_bond, wl.r0)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=50, k_bond=wl.k_bond,
                               r0_bond=wl.r0, excl_span=span), precision=precision, k_max=256)
    s.set_state(wl.x, types=wl.types)
    n = s.count().cpu().numpy()
    F, e, UW = s.force()
    s.check()
    print(f"[excl] {precision}: normwise {_normwise(F.cpu().numpy(), ref['F'] + Fb):.2e}", flush=True)
    assert np.abs(n - ref["n"]).max() <= (1e-12 if precision == "fp64" else 1e-5)
    assert _normwise(F.cpu().numpy(), ref["F"] + Fb) <= tol
    assert abs(UW[0, 0].item() - (ref["U"] + Ub)) <= tol * (np.abs(ref["e"]).sum() + Ub)
    # the list still holds every pair (exclusions only switch terms off)
    pairs, cnt = s.nlist_pairs(0)
    got = {(int(a), int(b)) for a, b in pairs if a < b}
    want = {tuple(p) for p in oracle.neighbor_pairs(wl.x, wl.L, 2.4).tolist()}
    assert got == want


def test_exclusion_trajectory_fp64():
    from paper_2609_07842_amd import vbc
    wl = W.polymer_melt(nchains=12, nbeads=20, seed=5, rho=0.6)
    span = 5
    bonds = wl.bonds
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=20, k_bond=wl.k_bond,
                               r0_bond=wl.r0, excl_span=span), precision="fp64", k_max=256)
    s.set_state(wl.x, wl.v, types=wl.types)
    s.step(30, integrator="langevin", dt=0.002, kT=1.0, gamma=0.5, seed=4)
    s.check()
    xg, vg = (t.cpu().numpy() for t in s.get_state())
    ref = oracle.run(wl.x, wl.v, wl.L, wl.params, 30, kind=oracle.LANGEVIN, dt=0.002, kT=1.0,
                     gamma=0.5, seed=4, types=wl.types, mask=wl.mask, bonds=bonds, k_bond=wl.k_bond,
                     r0=wl.r0, chain_len=20, excl_span=span)
    dx = xg - ref["x"]
    dx -= wl.L * np.rint(dx / wl.L)
    assert np.abs(dx).max() <= 1e-9 * wl.L
    assert np.abs(vg - ref["v"]).max() <= 1e-8 * max(1.0, np.abs(ref["v"]).max())
