"""Host-side logic of the request loop: pool layout derived from the request range and
footprints that grow with size (no GPU needed)."""
import numpy as np
import pytest

from paper_2609_07842_amd import workloads as W


def _lib_or_skip():
    try:
        from paper_2609_07842_amd import vbc
        vbc.lib()
        return vbc
    except ImportError as e:
        pytest.skip(str(e))


def test_layout_covers_every_request_size():
    vbc = _lib_or_skip()
    from paper_2609_07842_amd import serve
    cfg = serve.ServerConfig()
    lay = serve.layout_for(cfg)
    for q in W.serving_requests(n=64, seed=5):
        fp = vbc.footprint(serve.request_desc(q), cfg.precision)
        assert fp["k_max"] <= lay["k_max"]
        assert fp["stage_cap"] <= lay["stage_cap"]
        assert lay["bcap_min"] <= fp["bcap"] <= lay["bcap_max"]
        fp2 = vbc.footprint(serve.request_desc(q), cfg.precision, k_max=lay["k_max"],
                            stage_cap=lay["stage_cap"])
        assert fp2["bytes"] >= lay["bytes_per_slot"] * fp2["slots"] - 1e-6


def test_footprint_grows_with_size_and_list_length():
    vbc = _lib_or_skip()
    p = W.vbc_params()
    small = vbc.footprint(vbc.replica(1000, W.box_length(1000, 0.3), p), "fp32", k_max=56, stage_cap=1920)
    large = vbc.footprint(vbc.replica(100000, W.box_length(100000, 0.3), p), "fp32", k_max=56,
                          stage_cap=1920)
    longer = vbc.footprint(vbc.replica(100000, W.box_length(100000, 0.3), p), "fp32", k_max=112,
                           stage_cap=1920)
    assert small["bytes"] < large["bytes"] < longer["bytes"]
    # 7 more 16-byte list chunks per slot
    assert longer["bytes"] - large["bytes"] == 16 * 7 * large["slots"]
    assert large["slots"] >= 100000 and large["slots"] % large["bcap"] == 0


def test_poisson_arrivals_follow_the_stream_gaps():
    from paper_2609_07842_amd import serve
    reqs = W.serving_requests(n=256, seed=5)
    t = serve.poisson_arrivals(reqs, rate=50.0)
    assert np.all(np.diff(t) >= 0)
    assert t[-1] == pytest.approx(sum(q["gap"] for q in reqs) / 50.0)
    assert 256 / t[-1] == pytest.approx(50.0, rel=0.2)


def test_rho_max_sizes_the_layout_for_dense_regions():
    vbc = _lib_or_skip()
    p = W.vbc_params(f=3.0, E_a=5.0)
    d = vbc.replica(100_000, W.box_length(100_000, 0.3), p)
    a = vbc.footprint(d, "fp32")
    b = vbc.footprint(d, "fp32", rho_max=1.0)
    assert b["bcap"] > a["bcap"] and b["stage_cap"] > a["stage_cap"] and b["k_max"] > a["k_max"]
    # a brick of 4^3 cells of edge >= 2.4 at density 1.0 holds ~900 particles: they must fit
    assert b["bcap"] >= 1.0 * 64 * 2.4 ** 3
    # at rho_max below the mean density nothing changes
    c = vbc.footprint(d, "fp32", rho_max=0.1)
    assert c == a
