"""GPU clusters of the bond graph (Section 3) against the oracle, bit for bit: per particle
the smallest tag of its cluster, per replica the statistics (clusters, largest, particles in
cyclic clusters, bonds, cyclic clusters) and the size histograms of all and of acyclic
clusters.  The bond test is decided in FP64 the same way on both sides, so every integer
must agree exactly."""
import numpy as np
import pytest

import oracle
from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


def _check(lab, stats, hist, x, L, params, types=None, hist_len=64, large=False):
    fn = oracle.bond_clusters_large if large else oracle.bond_clusters
    lr, zr = fn(x, L, params, types)
    st = oracle.cluster_stats(lr, zr, hist_len)
    assert np.array_equal(lab, lr)
    assert list(stats) == [st["clusters"], st["largest"], st["cyclic_particles"], st["bonds"],
                           st["cyclic_clusters"]]
    assert np.array_equal(hist, st["hist"])
    return st


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("rho,f,E_a", [(0.05, 2.0, 6.0), (0.3, 4.0, 5.0)])
def test_clusters_bit_exact_along_a_trajectory(precision, rho, f, E_a):
    vbc = _vbc()
    wl = W.fluid(3000, rho, f, E_a=E_a, seed=5)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision=precision, rho_max=1.0)
    s.set_state(wl.x, wl.v)
    for k in range(3):
        if k:
            s.step(150, integrator="langevin", seed=3)
        lab, stats, hist = s.clusters(hist_len=64)
        s.check()
        x = s.get_state()[0].cpu().numpy()
        st = _check(lab.cpu().numpy(), stats.cpu().numpy()[0], hist.cpu().numpy()[0], x, wl.L, wl.params)
        print(f"[clusters] {precision} rho {rho} step {150 * k}: {st['clusters']} clusters, largest "
              f"{st['largest']}, x_cyc {st['cyclic_particles'] / wl.N:.3f}, bonds {st['bonds']}", flush=True)


def test_clusters_of_known_shapes_on_gpu():
    """The oracle's fixture of a ring, a chain, a tetrahedron and lone particles."""
    vbc = _vbc()
    import math
    pts = []
    for k in range(6):
        a = 2 * math.pi * k / 6
        pts.append([5 + 1.2 * math.cos(a), 5 + 1.2 * math.sin(a), 5.0])
    pts += [[15 + 1.2 * k, 15.0, 15.0] for k in range(4)]
    e = 1.2 / math.sqrt(8.0)
    pts += [[25 + e * a, 25 + e * b, 25 + e * c] for a, b, c in ((1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1))]
    pts += [[35.0, 5.0, 5.0], [5.0, 35.0, 35.0], [35.0, 35.0, 5.0]]
    x = np.array(pts)
    params = W.vbc_params()
    s = vbc.System(vbc.replica(len(x), 40.0, params), precision="fp64")
    s.set_state(x)
    lab, stats, hist = s.clusters(hist_len=8)
    s.check()
    assert lab.cpu().numpy().tolist() == [0] * 6 + [6] * 4 + [10] * 4 + [14, 15, 16]
    assert stats.cpu().numpy()[0].tolist() == [6, 6, 10, 15, 2]
    assert hist.cpu().numpy()[0].tolist() == [[0, 3, 0, 0, 2, 0, 1, 0], [0, 3, 0, 0, 1, 0, 0, 0]]


def test_clusters_in_a_pool_and_multitype():
    vbc = _vbc()
    a = W.fluid(1500, 0.1, 2.0, E_a=6.0, seed=1)
    b = W.fluid(2500, 0.4, 5.0, seed=2)
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
    lab, stats, hist = pool.clusters(hist_len=32)
    pool.check()
    lab, stats, hist = lab.cpu().numpy(), stats.cpu().numpy(), hist.cpu().numpy()
    for r, w in ((ra, a), (rb, b)):
        n, off = pool.info(r)
        _check(lab[off:off + n], stats[r], hist[r], np.mod(w.x, w.L), w.L, w.params, hist_len=32)
    assert (stats[3 - ra - rb] == 0).all() and (hist[3 - ra - rb] == 0).all()
    # two types with their own attraction ranges
    rng = np.random.default_rng(4)
    N = 2000
    L = W.box_length(N, 0.4)
    types = rng.integers(0, 2, size=N).astype(np.int32)
    pa = W.vbc_params(f=2.0)
    pb = dict(W.vbc_params(f=3.0), r_r=0.8, r_a=1.3, r_l=1.3, r_h=1.7)
    pab = dict(W.vbc_params(f=1.0), r_r=0.9, r_a=1.4, r_l=1.4, r_h=1.8)
    params = [pa, pab, pab, pb]
    x = np.mod(W.uniform_positions(N, L, 5), L)
    s = vbc.System(vbc.replica(N, L, params), precision="fp32")
    s.set_state(x, types=types)
    lab, stats, hist = s.clusters(hist_len=16)
    _check(lab.cpu().numpy(), stats.cpu().numpy()[0], hist.cpu().numpy()[0], x, L, params, types, hist_len=16)


def test_clusters_full_size_every_label():
    """N = 10^6 at density 0.5 (the headline workload) after 100 Langevin steps: every label,
    the statistics and the histogram against the k-d tree form of the oracle."""
    vbc = _vbc()
    wl = W.fluid(1_000_000, 0.5, 4.0, E_a=5.0, seed=7)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32")
    s.set_state(wl.x, wl.v)
    s.step(100, integrator="langevin", seed=1)
    lab, stats, hist = s.clusters(hist_len=4096)
    s.check()
    x = s.get_state()[0].cpu().numpy()
    st = _check(lab.cpu().numpy(), stats.cpu().numpy()[0], hist.cpu().numpy()[0], x, wl.L, wl.params,
                hist_len=4096, large=True)
    print(f"[clusters] N=1e6: {st['clusters']} clusters, P_inf {st['largest'] / wl.N:.4f}", flush=True)
