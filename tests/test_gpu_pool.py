"""GPU tests of replica pools (continuous batching): replicas admitted into and retired
from a fixed-capacity pool while others keep running give, bit for bit, the results
they give alone; pool forces and Langevin trajectories match the oracle; whole-call step
graphs give the same bits as individual launches; capacity limits are reported; every
step leaves one time stamp."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# list and staging capacity that covers densities up to 0.5 with the standard geometry
OPTS = dict(k_max=72, stage_cap=2112, block=256)


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


def _normwise(a, b):
    return np.linalg.norm(np.asarray(a) - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300)


def _requests():
    """Four replicas of different size, density, valency and well depth."""
    out = []
    for k, (N, rho, f, E_a) in enumerate([(700, 0.3, 2.0, 5.0), (1500, 0.5, 4.0, 3.0),
                                          (400, 0.15, 1.0, 8.0), (2600, 0.3, 6.0, 2.0)]):
        L = W.box_length(N, rho)
        out.append(dict(N=N, L=L, p=W.vbc_params(E_a=E_a, f=f), x=W.uniform_positions(N, L, 60 + k),
                        v=W.maxwell_boltzmann(N, 1.0, 70 + k), seed=1000 + 17 * k))
    return out


def _desc(vbc, m):
    return vbc.replica(m["N"], m["L"], m["p"], seed=m["seed"])


def _pool(vbc, precision, reqs, max_replicas=6, slack=2.0):
    fps = [vbc.footprint(_desc(vbc, m), precision, **OPTS) for m in reqs]
    caps = dict(max_replicas=max_replicas, max_types=1,
                max_particles=int(slack * sum(m["N"] for m in reqs)),
                max_slots=int(slack * sum(f["slots"] for f in fps)),
                max_bricks=int(slack * sum(f["bricks"] for f in fps)),
                max_cells=int(slack * sum(f["cells"] for f in fps)),
                max_bcap=max(f["bcap"] for f in fps), chains=False)
    return vbc.Pool(caps, precision=precision, **OPTS)


def _state(sysm, rep):
    x, v = sysm.get_state(rep)
    return x.cpu().numpy(), v.cpu().numpy()


LANG = dict(integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_staggered_admission_equals_alone_bitwise(precision):
    """Admit A, run, admit B, run, admit C, run, retire A, admit D into the freed ranges,
    run: every replica ends bit-identical to running it alone with the same calls."""
    vbc = _vbc()
    A, B, C, D = _requests()
    print(f"[pool staggered] {precision}", flush=True)
    pool = _pool(vbc, precision, [A, B, C, D])
    ra = pool.admit(_desc(vbc, A), A["x"], A["v"])
    pool.step(16, **LANG)
    rb = pool.admit(_desc(vbc, B), B["x"], B["v"])
    pool.step(16, **LANG)
    rc = pool.admit(_desc(vbc, C), C["x"], C["v"])
    pool.step(8, **LANG)
    xa, va = _state(pool, ra)
    pool.retire(ra)
    pool.step(16, **LANG)
    rd = pool.admit(_desc(vbc, D), D["x"], D["v"])
    assert rd == ra  # the first free slot is reused
    pool.step(16, **LANG)
    pool.check()
    got = {"A": (xa, va), "B": _state(pool, rb), "C": _state(pool, rc), "D": _state(pool, rd)}
    calls = {"A": [16, 16, 8], "B": [16, 8, 16, 16], "C": [8, 16, 16], "D": [16]}
    for name, m in zip("ABCD", (A, B, C, D)):
        alone = _pool(vbc, precision, [m], max_replicas=1)
        r = alone.admit(_desc(vbc, m), m["x"], m["v"])
        for n in calls[name]:
            alone.step(n, **LANG)
        alone.check()
        x1, v1 = _state(alone, r)
        assert np.array_equal(x1, got[name][0]), name
        assert np.array_equal(v1, got[name][1]), name


def test_pool_matches_fixed_set_bitwise():
    """A replica in a pool and the same replica in a vbc_create handle with the same
    options give the same forces, energies and trajectory bits."""
    vbc = _vbc()
    reqs = _requests()[:3]
    pool = _pool(vbc, "fp32", reqs)
    slots = [pool.admit(_desc(vbc, m), m["x"], m["v"]) for m in reqs]
    F, e, UW = pool.force()
    F, e, UW = F.cpu().numpy(), e.cpu().numpy(), UW.cpu().numpy()
    pool.step(24, **LANG)
    pool.check()
    for m, r in zip(reqs, slots):
        n, off = pool.info(r)
        assert n == m["N"]
        s = vbc.System(_desc(vbc, m), precision="fp32", **OPTS)
        s.set_state(m["x"], m["v"])
        F1, e1, UW1 = s.force()
        assert np.array_equal(F1.cpu().numpy(), F[off:off + n])
        assert np.array_equal(e1.cpu().numpy(), e[off:off + n])
        assert np.array_equal(UW1.cpu().numpy()[0], UW[r])
        s.step(24, **LANG)
        s.check()
        x1, v1 = _state(s, 0)
        x2, v2 = _state(pool, r)
        assert np.array_equal(x1, x2) and np.array_equal(v1, v2)


def test_pool_forces_match_oracle_after_reuse():
    """FP64 pool: after a retire and a re-admission into the freed ranges, the new
    replica's forces, energies and virial match the oracle."""
    vbc = _vbc()
    A, B, C, D = _requests()
    pool = _pool(vbc, "fp64", [A, B, D], max_replicas=3)
    ra = pool.admit(_desc(vbc, A), A["x"], A["v"])
    rb = pool.admit(_desc(vbc, B), B["x"], B["v"])
    pool.step(10, **LANG)
    pool.retire(ra)
    rd = pool.admit(_desc(vbc, D), D["x"], None)
    F, e, UW = pool.force()
    n, off = pool.info(rd)
    ref = oracle.evaluate(D["x"], D["L"], D["p"])
    assert _normwise(F.cpu().numpy()[off:off + n], ref["F"]) <= 1e-10
    assert abs(UW.cpu().numpy()[rd, 0] - ref["U"]) <= 1e-10 * max(1.0, abs(ref["U"]))
    assert abs(UW.cpu().numpy()[rd, 1] - ref["W"]) <= 1e-10 * max(1.0, abs(ref["W"]))
    # the replica that kept running still has its own particles and finite forces
    nb, offb = pool.info(rb)
    assert nb == B["N"]
    assert np.isfinite(F.cpu().numpy()[offb:offb + nb]).all()


def test_replica_seed_keys_the_noise():
    """FP64 Langevin in a pool: a replica with seed s under integrator seed k follows the
    oracle's trajectory with noise key k + s."""
    vbc = _vbc()
    wl = W.small_fluid(N=300)
    m = dict(N=wl.N, L=wl.L, p=wl.params, x=wl.x, v=wl.v, seed=123456789)
    other = _requests()[2]
    pool = _pool(vbc, "fp64", [m, other], max_replicas=2)
    pool.admit(_desc(vbc, other), other["x"], other["v"])
    r = pool.admit(_desc(vbc, m), m["x"], m["v"])
    pool.step(30, **LANG)
    pool.check()
    x, v = _state(pool, r)
    ref = oracle.run(wl.x, wl.v, wl.L, wl.params, 30, kind=oracle.LANGEVIN, dt=0.005, kT=1.0,
                     gamma=0.1, seed=LANG["seed"] + m["seed"])
    dx = x - ref["x"]
    dx -= wl.L * np.rint(dx / wl.L)
    assert np.abs(dx).max() <= 1e-9 * wl.L
    assert np.abs(v - ref["v"]).max() <= 1e-9 * max(1.0, np.abs(ref["v"]).max())


def test_call_graph_equals_individual_launches():
    """Whole-call graphs (kernel timing off) and individual launches (timing on) give
    the same bits."""
    vbc = _vbc()
    reqs = _requests()[:2]
    out = []
    for timing in (False, True):
        pool = _pool(vbc, "fp32", reqs)
        slots = [pool.admit(_desc(vbc, m), m["x"], m["v"]) for m in reqs]
        if timing:
            pool.profile(True, 4096)
        for _ in range(3):
            pool.step(12, **LANG)
        pool.check()
        out.append([_state(pool, r) for r in slots])
    for (x0, v0), (x1, v1) in zip(*out):
        assert np.array_equal(x0, x1) and np.array_equal(v0, v1)


def test_capacity_limits_are_reported():
    vbc = _vbc()
    A, B, C, D = _requests()
    pool = _pool(vbc, "fp32", [A, C], max_replicas=2, slack=1.0)
    pool.admit(_desc(vbc, A), A["x"])
    with pytest.raises(vbc.VBCError) as ei:  # more particle slots than are left
        pool.admit(_desc(vbc, D), D["x"])
    assert ei.value.status == vbc.VBC_ERR_CAPACITY
    pool.admit(_desc(vbc, C), C["x"])
    with pytest.raises(vbc.VBCError) as ei:  # no replica slot left
        pool.admit(_desc(vbc, C), C["x"])
    assert ei.value.status == vbc.VBC_ERR_CAPACITY
    with pytest.raises(vbc.VBCError) as ei:  # too dense for the pool's list length
        dense = W.box_length(500, 0.9)
        pool2 = _pool(vbc, "fp32", [A])
        pool2.admit(vbc.replica(500, dense, W.vbc_params()), W.uniform_positions(500, dense, 3))
    assert ei.value.status == vbc.VBC_ERR_CAPACITY
    with pytest.raises(vbc.VBCError) as ei:
        pool.retire(5)
    assert ei.value.status == vbc.VBC_ERR_ARG


def test_step_stamps():
    vbc = _vbc()
    reqs = _requests()[:2]
    pool = _pool(vbc, "fp32", reqs)
    for m in reqs:
        pool.admit(_desc(vbc, m), m["x"], m["v"])
    pool.step(4, **LANG)
    pool.stamps(True)
    for _ in range(3):
        pool.step(10, **LANG)
    t = pool.stamps_read()
    assert len(t) == 30
    d = np.diff(t)
    assert (d > 0).all() and d.max() < 0.1
    pool.stamps(False)
    pool.step(5, **LANG)
    assert len(pool.stamps_read()) == 0
