"""vbc_clusters_noalloc (the cluster analysis with the library's own fixed scratch, for
callers that cannot allocate) against vbc_clusters with caller scratch on the same handles:
every label, statistic and histogram bin identical, on two calls in a row, the second on a
smaller system, so that it runs over what the first left in the shared array."""
import numpy as np
import pytest

from paper_2609_07842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vbc():
    from paper_2609_07842_amd import vbc
    return vbc


def _fluid(vbc, N, rho, f, seed, steps):
    wl = W.fluid(N, rho, f, E_a=5.0, seed=seed)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp32", rho_max=1.0)
    s.set_state(wl.x, wl.v)
    if steps:
        s.step(steps, integrator="langevin", seed=seed)
    return s


def test_noalloc_clusters_equal_caller_scratch():
    vbc = _vbc()
    big = _fluid(vbc, 20000, 0.3, 4.0, seed=21, steps=200)
    small = _fluid(vbc, 1500, 0.1, 2.0, seed=22, steps=50)
    print("[noalloc] two calls: N=20000, then N=1500", flush=True)
    out_big = big.clusters_noalloc(hist_len=128)
    out_small = small.clusters_noalloc(hist_len=32)
    big.check()
    small.check()
    for s, got, hl in ((big, out_big, 128), (small, out_small, 32)):
        ref = s.clusters(hist_len=hl)
        s.check()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        st = got[1].cpu().numpy()[0]
        assert st[0] >= 1 and st[1] >= 1  # clusters found, largest non-empty
    # the same handle again after the smaller one: still identical
    again = big.clusters_noalloc(hist_len=128)
    for a, b in zip(again, out_big):
        assert torch.equal(a, b)
    big.close()
    small.close()


def test_noalloc_clusters_reject_handles_beyond_the_fixed_scratch():
    vbc = _vbc()
    N = 1_200_000  # about 1.9 x 10^6 particle slots at density 0.5: above the fixed scratch
    L = W.box_length(N, 0.5)
    s = vbc.System(vbc.replica(N, L, W.vbc_params(E_a=5.0, f=4.0)), precision="fp32")
    with pytest.raises(vbc.VBCError) as ei:
        s.clusters_noalloc(hist_len=16)
    assert ei.value.status == vbc.VBC_ERR_CAPACITY
    s.close()
