"""GPU tests of the per-step energy and virial (vbc_thermo) and of capturing the step
graphs ahead of a call (vbc_step_prepare): the last step's energy and virial against the
oracle at the GPU's final positions, the sums over steps against the oracle's trajectory,
a replica's sums alone and in a pool bit for bit, the sums independent of how the steps are
split into calls, and prepared calls bit for bit equal to unprepared ones."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


def _min_image(d, L):
    return d - L * np.rint(d / L)


@pytest.mark.parametrize("case", ["small", "window_mid"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_thermo_matches_oracle(precision, tol, case):
    vbc = _vbc()
    # small: N = 1000 at density 0.3, f = 2; window_mid: N = 4000 at density 0.5, f = 6,
    # where tens of particles per brick sit in a switching window (chain-rule terms)
    wl = W.small_fluid() if case == "small" else W.small_fluid(N=4000, rho=0.5, f=6.0)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision=precision)
    s.set_state(wl.x, wl.v)
    s.thermo(True)
    nsteps = 30
    s.step(nsteps, integrator="nve", dt=0.005)
    th = s.thermo_read()[0]
    s.check()
    assert th["steps"] == nsteps
    x = s.get_state()[0].cpu().numpy()
    ref = oracle.evaluate(x, wl.L, wl.params)
    scale = np.abs(ref["e"]).sum()
    want = np.concatenate([[ref["U"], ref["W"]], ref["Wt"]])
    print(f"[thermo {precision}] last {th['last'][:2]} oracle {want[:2]}", flush=True)
    assert np.abs(th["last"] - want).max() <= tol * (scale + np.abs(want).max())
    # the sum of U over the steps against the oracle's trajectory (FP64 only: the FP32
    # trajectory drifts from the exact one by more than the energies' tolerance)
    if precision == "fp64":
        run = oracle.run(wl.x, wl.v, wl.L, wl.params, nsteps, kind=oracle.NVE, dt=0.005, history=True)
        assert abs(th["sum"][0] - run["U"].sum()) <= 1e-9 * np.abs(run["U"]).sum()
    # read clears; off stops the sums
    assert s.thermo_read()[0]["steps"] == 0
    s.thermo(False)
    s.step(4, integrator="nve", dt=0.005)
    assert s.thermo_read()[0]["steps"] == 0
    s.close()


def test_thermo_alone_and_in_a_pool_bitwise():
    vbc = _vbc()
    opts = dict(k_max=72, stage_cap=2400, block=256)
    a = W.fluid(1200, 0.3, 2.0, E_a=5.0, seed=31)
    b = W.fluid(2500, 0.4, 4.0, E_a=3.0, seed=32)
    da = vbc.replica(a.N, a.L, a.params, seed=7)
    db = vbc.replica(b.N, b.L, b.params, seed=9)
    integ = dict(integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=5)
    fps = [vbc.footprint(d, "fp32", **opts) for d in (da, db)]
    caps = dict(max_replicas=4, max_types=1, max_particles=2 * (a.N + b.N),
                max_slots=2 * sum(f["slots"] for f in fps), max_bricks=2 * sum(f["bricks"] for f in fps),
                max_cells=2 * sum(f["cells"] for f in fps), max_bcap=max(f["bcap"] for f in fps),
                chains=False)
    alone = vbc.Pool(caps, precision="fp32", **opts)
    ra = alone.admit(da, a.x, a.v)
    alone.thermo(True)
    alone.step(24, **integ)
    t_alone = alone.thermo_read()[ra]
    alone.check()
    alone.close()
    mix = vbc.Pool(caps, precision="fp32", **opts)
    rb = mix.admit(db, b.x, b.v)
    ra = mix.admit(da, a.x, a.v)
    mix.thermo(True)
    mix.step(24, **integ)
    t_mix = mix.thermo_read()
    mix.check()
    mix.close()
    assert t_mix[ra]["steps"] == 24 and t_mix[rb]["steps"] == 24
    assert np.array_equal(t_alone["last"], t_mix[ra]["last"])
    assert np.array_equal(t_alone["sum"], t_mix[ra]["sum"])


def test_thermo_sums_do_not_depend_on_the_call_split():
    # a step's sums are added by the next step's count pass, the call's last step's by the
    # closing reduction: both must give the same bits, so one call of 90 steps (graphs of
    # eight steps), three of 30 (whole-call graphs) and 90 of one step agree exactly
    vbc = _vbc()
    wl = W.fluid(2000, 0.4, 3.0, E_a=5.0, seed=34)
    integ = dict(integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=6)
    res = []
    for split in ([90], [30, 30, 30], [1] * 90):
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32", block=256)
        s.set_state(wl.x, wl.v)
        s.thermo(True)
        for n in split:
            s.step(n, **integ)
        th = s.thermo_read()[0]
        s.check()
        res.append((th["steps"], th["last"], th["sum"]))
        s.close()
    for steps, last, sums in res[1:]:
        assert steps == res[0][0] == 90
        assert np.array_equal(last, res[0][1])
        assert np.array_equal(sums, res[0][2])


@pytest.mark.parametrize("nsteps", [20, 100])
def test_prepared_call_equals_unprepared(nsteps):
    vbc = _vbc()
    wl = W.fluid(3000, 0.4, 3.0, E_a=5.0, seed=33)
    integ = dict(integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=8)
    out = []
    for prepare in (False, True):
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32")
        s.set_state(wl.x, wl.v)
        s.step(3, **integ)
        if prepare:
            s.prepare_step(nsteps, **integ)
            s.prepare_step(nsteps, **integ)  # a second capture of the same shape is a no-op
        s.step(nsteps, **integ)
        s.check()
        out.append([t.cpu().numpy() for t in s.get_state()])
        s.close()
    for u, w in zip(out[0], out[1]):
        assert np.array_equal(u, w)
