"""GPU tests of the systems around the passes: several replicas in one handle (each
result bitwise identical to running it alone), per-replica state replacement,
checkpoint/resume bit-identity, error reporting forced from the host, a bead-spring melt
with sticker types and bonds, and sampled parity at 10^5 and 10^6 particles."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


def _normwise(a, b):
    return np.linalg.norm(np.asarray(a) - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300)


def _mix():
    out = []
    for k, (N, rho, f, E_a) in enumerate([(700, 0.3, 2.0, 5.0), (1500, 0.5, 4.0, 3.0),
                                          (400, 0.15, 1.0, 8.0)]):
        L = W.box_length(N, rho)
        out.append(dict(N=N, L=L, p=W.vbc_params(E_a=E_a, f=f), x=W.uniform_positions(N, L, 40 + k),
                        v=W.maxwell_boltzmann(N, 1.0, 50 + k)))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_replicas_alone_equal_mixed_bitwise(precision):
    vbc = _vbc()
    mix = _mix()
    print(f"[mix] {precision}", flush=True)
    big = vbc.System([vbc.replica(m["N"], m["L"], m["p"]) for m in mix], precision=precision)
    big.set_state(np.concatenate([m["x"] for m in mix]), np.concatenate([m["v"] for m in mix]))
    Fb, eb, UWb = big.force()
    big.step(60, integrator="langevin", seed=7)
    big.check()
    xb, vb = big.get_state()
    xb, vb, Fb = xb.cpu().numpy(), vb.cpu().numpy(), Fb.cpu().numpy()
    off = 0
    for k, m in enumerate(mix):
        s = vbc.System(vbc.replica(m["N"], m["L"], m["p"]), precision=precision)
        s.set_state(m["x"], m["v"])
        F1, e1, UW1 = s.force()
        s.step(60, integrator="langevin", seed=7)
        s.check()
        x1, v1 = s.get_state()
        sl = slice(off, off + m["N"])
        assert np.array_equal(F1.cpu().numpy(), Fb[sl])
        assert np.array_equal(UW1.cpu().numpy()[0], UWb.cpu().numpy()[k])
        assert np.array_equal(x1.cpu().numpy(), xb[sl])
        assert np.array_equal(v1.cpu().numpy(), vb[sl])
        off += m["N"]


def test_set_state_of_one_replica_leaves_others_running():
    vbc = _vbc()
    mix = _mix()
    big = vbc.System([vbc.replica(m["N"], m["L"], m["p"]) for m in mix], precision="fp64")
    big.set_state(np.concatenate([m["x"] for m in mix]), np.concatenate([m["v"] for m in mix]))
    big.step(20, integrator="nve")
    # replace replica 1 by a fresh configuration; 0 and 2 continue
    fresh = W.uniform_positions(mix[1]["N"], mix[1]["L"], 99)
    big.set_state(fresh, None, rep=1)
    big.step(20, integrator="nve")
    big.check()
    x, v = big.get_state()
    x = x.cpu().numpy()
    # replica 0 alone for 40 steps
    m = mix[0]
    s = vbc.System(vbc.replica(m["N"], m["L"], m["p"]), precision="fp64")
    s.set_state(m["x"], m["v"])
    s.step(20, integrator="nve")
    s.step(20, integrator="nve")
    x0, _ = s.get_state()
    assert np.abs(x0.cpu().numpy() - x[: m["N"]]).max() < 1e-12
    # replica 1 from the fresh start for 20 steps, against the oracle
    ref = oracle.run(fresh, np.zeros_like(fresh), mix[1]["L"], mix[1]["p"], 20, kind=oracle.NVE)
    d = x[mix[0]["N"]: mix[0]["N"] + mix[1]["N"]] - ref["x"]
    d -= mix[1]["L"] * np.rint(d / mix[1]["L"])
    assert np.abs(d).max() < 1e-9


def test_checkpoint_resume_bitwise():
    vbc = _vbc()
    wl = W.small_fluid(N=1200, rho=0.4, f=3.0)
    a = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32")
    a.set_state(wl.x, wl.v)
    a.step(50, integrator="langevin", seed=3)
    xc, vc = (t.cpu().numpy().copy() for t in a.get_state())
    a.build_nlist()  # a checkpoint is a list-build point
    a.step(50, integrator="langevin", seed=3)
    xa, va = (t.cpu().numpy() for t in a.get_state())
    b = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32")
    b.set_state(xc, vc, step0=50)
    b.step(50, integrator="langevin", seed=3)
    xb, vb = (t.cpu().numpy() for t in b.get_state())
    a.check()
    b.check()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)


def test_kernel_timing_leaves_the_trajectory_and_times_every_pass():
    """The timing mode launches each pass through hipExtLaunchKernel with a pair of events
    that its dispatches record: same bits as the step graphs, one timed launch per pass and
    step, and per-pass times that fit inside the wall time of the steps."""
    import time
    vbc = _vbc()
    wl = W.small_fluid(N=3000, rho=0.5, f=4.0)
    out = []
    for timing in (False, True):
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32")
        s.set_state(wl.x, wl.v)
        s.step(20, integrator="langevin", seed=5)
        if timing:
            s.profile(True, 1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(40, integrator="langevin", seed=5)
        torch.cuda.synchronize()
        wall_ms = 1e3 * (time.perf_counter() - t0)
        s.check()
        out.append([t.cpu().numpy().copy() for t in s.get_state()])
        if timing:
            prof = s.profile_read()
            print(f"[timing] wall {wall_ms:.3f} ms, " +
                  ", ".join(f"{k} {v[0]:.3f} ms/{v[1]}" for k, v in prof.items()), flush=True)
            for k in ("build", "count", "embed", "force"):
                assert prof[k][1] == 40, (k, prof[k])
                assert prof[k][0] > 0.0, (k, prof[k])
            assert sum(prof[k][0] for k in ("build", "count", "embed", "force")) <= wall_ms
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_stage_capacity_overflow_reported():
    vbc = _vbc()
    N = 3000
    L = W.box_length(N, 0.5)
    s = vbc.System(vbc.replica(N, L, W.vbc_params()), precision="fp32", stage_cap=256)
    s.set_state(W.uniform_positions(N, L, 1))
    s.force()
    st, flags = s.check(raise_on_error=False)
    assert st == vbc.VBC_ERR_CAPACITY


def test_resort_after_overflowed_build_keeps_every_particle():
    """A re-sort after a list build that overflowed the staging capacity cannot read its
    candidates through that build's staging map and walks the cell tables instead: every
    particle keeps its position (read back unchanged) and the overflow stays reported."""
    vbc = _vbc()
    N = 3000
    L = W.box_length(N, 0.5)
    x = W.uniform_positions(N, L, 1)
    s = vbc.System(vbc.replica(N, L, W.vbc_params()), precision="fp32", stage_cap=256)
    s.set_state(x)
    s.build_nlist()  # the full build from caller order: overflows
    s.build_nlist()  # an incremental build: re-sort, then list
    st, flags = s.check(raise_on_error=False)
    assert st == vbc.VBC_ERR_CAPACITY
    xs, _ = s.get_state()
    np.testing.assert_array_equal(xs.cpu().numpy(), x)


def test_lost_particle_reported():
    vbc = _vbc()
    N = 2000
    L = W.box_length(N, 0.3)
    x = W.uniform_positions(N, L, 2)
    v = np.zeros((N, 3))
    v[5] = [2000.0, 0.0, 0.0]  # 10 length units in one step of 0.005: a jump of several cells
    s = vbc.System(vbc.replica(N, L, W.vbc_params(E_r=0.0, E_a=0.0)), precision="fp64")
    s.set_state(x, v)
    s.step(2, integrator="nve", dt=0.005)
    st, flags = s.check(raise_on_error=False)
    assert st == vbc.VBC_ERR_NONFINITE
    assert flags[0] & vbc.FLAG_LOST


def test_polymer_melt_parity():
    """Bead-spring melt (40 chains x 50 beads at density 0.85, harmonic bonds k = 100,
    every fifth bead a valency-1 sticker with well depth 8 counting only stickers) against
    the oracle's VBC evaluation plus its bond forces."""
    vbc = _vbc()
    wl = W.polymer_melt(nchains=40, nbeads=50, seed=7)
    ref = oracle.evaluate(wl.x, wl.L, wl.params, wl.types, wl.mask)
    Ub, Fb, Wb = oracle.bonds_energy_forces(wl.x, wl.L, wl.bonds, wl.k_bond, wl.r0, virial=True)
    Fref = ref["F"] + Fb
    # {W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz} of pair terms plus bonds
    Wref = np.concatenate([[ref["W"]], ref["Wt"]]) + Wb
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        print(f"[melt] {prec}", flush=True)
        # random-walk starts pack beads at bond distance: size the list for that
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=50,
                                   k_bond=wl.k_bond, r0_bond=wl.r0), precision=prec, k_max=256)
        s.set_state(wl.x, types=wl.types)
        n = s.count().cpu().numpy()
        F, e, UW = s.force()
        s.check()
        assert np.abs(n - ref["n"]).max() <= (1e-12 if prec == "fp64" else 1e-5)
        assert _normwise(F.cpu().numpy(), Fref) <= tol
        assert abs(UW[0, 0].item() - (ref["U"] + Ub)) <= tol * (np.abs(ref["e"]).sum() + Ub)
        wscale = np.abs(Wref).max() + np.abs(ref["e"]).sum() + Ub
        assert np.abs(UW[0, 1:8].cpu().numpy() - Wref).max() <= tol * wscale


@pytest.mark.parametrize("N,rho,f,nsample",
                         [(100_000, 0.3, float(f), 48) for f in range(1, 7)] + [(1_000_000, 0.5, 4.0, 24)])
def test_sampled_parity_at_full_size(N, rho, f, nsample):
    """Full-size systems in the benchmark's launch configuration (FP32 pair arithmetic):
    forces and counts of sampled particles against the oracle's local evaluation, plus
    size-independent properties (net force, energy = sum of per-particle energies)."""
    vbc = _vbc()
    print(f"[sampled] N={N} f={f}", flush=True)
    wl = W.fluid(N, rho, f, E_a=5.0, seed=17)
    s = vbc.System(vbc.replica(N, wl.L, wl.params), precision="fp32")
    s.set_state(wl.x)
    n = s.count().cpu().numpy()
    F, e, UW = s.force()
    s.check()
    F = F.cpu().numpy()
    e = e.cpu().numpy()
    idx = np.random.default_rng(5).choice(N, size=nsample, replace=False)
    ref = oracle.evaluate_subset(wl.x, wl.L, wl.params, idx)
    assert np.abs(n[idx] - ref["n"]).max() <= 1e-5
    err = np.linalg.norm(F[idx] - ref["F"], axis=1).max() / np.linalg.norm(F, axis=1).max()
    print(f"  sampled normwise force error {err:.2e}", flush=True)
    assert err <= 1e-5
    assert np.abs(e[idx] - ref["e"]).max() <= 1e-5 * max(1.0, np.abs(e).max())
    assert abs(UW[0, 0].item() - e.sum()) <= 1e-9 * np.abs(e).sum()
    assert np.abs(F.sum(axis=0)).max() <= 1e-5 * np.linalg.norm(F, axis=1).max() * np.sqrt(N)


@pytest.mark.parametrize("f,steps,rho_max", [(4.0, 500, 0.0), (6.0, 2000, 0.9)])
def test_sampled_parity_headline_after_steps(f, steps, rho_max):
    """The headline fluid (N = 10^6, density 0.5, f = 4, FP32 pair arithmetic) after 500
    Langevin steps of its benchmark trajectory, in the benchmark's launch configuration,
    and the same fluid at f = 6 after 2000 steps (condensing, several per cent of the
    particles in a switching window; laid out for local densities up to 0.9 as in the
    valency sweep): counts and forces of particles inside a switching window (their counts
    are summed again in FP64), of their neighbours and of uniformly drawn particles against
    the oracle's local evaluation at the GPU's own positions."""
    from scipy.spatial import cKDTree
    vbc = _vbc()
    print(f"[sampled headline f={f:g} after {steps} steps] N=1000000", flush=True)
    wl = W.headline(f=f)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, skin=W.SKIN), precision="fp32",
                   **({"rho_max": rho_max} if rho_max else {}))
    s.set_state(wl.x, wl.v)
    s.step(steps, integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=3)
    s.check()
    x = s.get_state()[0].cpu().numpy()
    n = s.count().cpu().numpy()
    F, e, UW = s.force()
    s.check()
    F = F.cpu().numpy()
    x1 = wl.params["f"] - wl.params["delta"]
    rng = np.random.default_rng(29)
    win = np.nonzero((n > x1) & (n < x1 + 1.0))[0]
    print(f"  {len(win)} particles inside the switching window", flush=True)
    assert len(win) > 0
    pick = rng.choice(win, size=min(16, len(win)), replace=False)
    nb = set()
    for row in cKDTree(x, boxsize=wl.L).query_ball_point(x[pick], 2.0):
        nb.update(row)
    nb = np.array(sorted(nb - set(pick.tolist())), dtype=np.int64)
    nbs = rng.choice(nb, size=min(16, len(nb)), replace=False)
    uni = rng.choice(wl.N, size=16, replace=False)
    idx = np.unique(np.concatenate([pick, nbs, uni]))
    ref = oracle.evaluate_subset(x, wl.L, wl.params, idx)
    assert np.abs(n[idx] - ref["n"]).max() <= 1e-5
    w = np.isin(idx, pick)
    assert np.abs(n[idx][w] - ref["n"][w]).max() <= 1e-12
    assert np.any(ref["n"][w] > x1)
    err = np.linalg.norm(F[idx] - ref["F"], axis=1).max() / np.linalg.norm(F, axis=1).max()
    err_w = np.linalg.norm(F[idx][w] - ref["F"][w], axis=1).max() / np.linalg.norm(F, axis=1).max()
    print(f"  sampled normwise force error {err:.2e} (window particles {err_w:.2e})", flush=True)
    assert err <= 1e-5
    assert np.abs(F.sum(axis=0)).max() <= 1e-5 * np.linalg.norm(F, axis=1).max() * np.sqrt(wl.N)


def test_sampled_melt_parity_at_full_size():
    """The full bead-spring melt (20,000 chains x 50 beads = 10^6 beads at density 0.85,
    stickers every fifth bead) at its random-walk start, in the launch configuration the
    benchmark starts it in (FP32 pair arithmetic, bricks of 3^3 cells, k_max 256, sized for
    local densities up to 2): counts and forces (pair plus bond terms) of sampled beads
    against the oracle's local evaluation, and the net force."""
    vbc = _vbc()
    print("[sampled melt] N=1000000", flush=True)
    wl = W.polymer_melt(seed=4)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=50,
                               k_bond=wl.k_bond, r0_bond=wl.r0, skin=W.SKIN),
                   precision="fp32", brick=3, k_max=256, rho_max=2.0)
    s.set_state(wl.x, types=wl.types)
    n = s.count().cpu().numpy()
    F, e, UW = s.force()
    s.check()
    F = F.cpu().numpy()
    idx = np.random.default_rng(11).choice(wl.N, size=24, replace=False)
    ref = oracle.evaluate_subset(wl.x, wl.L, wl.params, idx, wl.types, wl.mask)
    _, Fb = oracle.bonds_energy_forces(wl.x, wl.L, wl.bonds, wl.k_bond, wl.r0)
    Fref = ref["F"] + Fb[idx]
    assert np.abs(n[idx] - ref["n"]).max() <= 1e-5
    err = np.linalg.norm(F[idx] - Fref, axis=1).max() / np.linalg.norm(F, axis=1).max()
    print(f"  sampled normwise force error {err:.2e}", flush=True)
    assert err <= 1e-5
    assert np.abs(F.sum(axis=0)).max() <= 1e-5 * np.linalg.norm(F, axis=1).max() * np.sqrt(wl.N)
