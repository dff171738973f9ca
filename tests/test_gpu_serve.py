"""GPU test of the continuous-batching request loop: requests that arrive while others
run are admitted as slots free up, run in one pool, and each one's final state is bit
for bit the state it reaches when served alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_served_mix_equals_alone_bitwise():
    from paper_2609_07842_amd import serve

    cfg = serve.ServerConfig(budget_bytes=48 << 20, max_replicas=3, max_particles=9000,
                             n_range=(1000, 4000), steps_per_tick=8, max_inflight=3)
    reqs = serve.make_requests(n=7, seed=9, rho=0.3, steps=48, n_range=(1000, 4000))
    print("[serve] sizes", [q["N"] for q in reqs], flush=True)
    srv = serve.Server(cfg)
    arrivals = serve.poisson_arrivals(reqs, rate=4000.0)  # arrivals overlap running requests
    mix = srv.run(reqs, arrivals, keep_results=True)
    assert mix["flagged"] == [] and mix["failed"] == 0
    assert mix["mean_live"] > 1.5                     # requests really ran together
    assert mix["queue_wait_s"]["p99"] > 0.0           # and admission made some wait
    assert mix["step_latency_ms"]["n"] == sum(q["steps"] - 1 for q in reqs)
    for k, q in enumerate(reqs):
        solo = srv.run([q], keep_results=True)
        x0, v0 = mix["results"][k]
        x1, v1 = solo["results"][0]
        assert torch.equal(x0, x1) and torch.equal(v0, v1), f"request {k}"


def test_overflowing_request_is_evicted_and_rerun():
    """A request whose particles start packed into half of its box (local density twice the
    layout's) overflows the main pool's brick capacity at its first list build.  The
    latched overflow flag is read while the others run; the request is evicted and run
    again from its initial state in the dense pool; every other request ends bit for bit
    where it ends alone, the re-run one where it ends alone, and nothing failed."""
    from paper_2609_07842_amd import serve
    from paper_2609_07842_amd import vbc

    cfg = serve.ServerConfig(budget_bytes=48 << 20, max_replicas=3, max_particles=9000,
                             n_range=(1000, 4000), steps_per_tick=8, max_inflight=3, check_every=2,
                             dense_budget_bytes=96 << 20, dense_max_replicas=2, dense_max_particles=9000)
    reqs = serve.make_requests(n=5, seed=9, rho=0.3, steps=48, n_range=(1000, 4000))
    bad = 2
    q = reqs[bad]
    L = float(serve.request_desc(q)["L"][0])
    x = q["x"].clone()
    x[:, 2] = x[:, 2] * 0.5  # every particle in the lower half of the box along z
    q["x"] = x
    print("[serve evict] sizes", [r["N"] for r in reqs], "packed request", bad, flush=True)
    srv = serve.Server(cfg)
    arrivals = serve.poisson_arrivals(reqs, rate=4000.0)
    mix = srv.run(reqs, arrivals, keep_results=True)
    print("[serve evict] flag events", mix["flagged"], flush=True)
    assert mix["failed"] == 0 and mix["completed"] == len(reqs)
    assert mix["flagged_in_figures"] == 0
    ev = [f for f in mix["flagged"] if f[0] == bad]
    assert ev and ev[0][1] == "main" and ev[0][2] & vbc.FLAG_STAGE_OVERFLOW
    assert mix["lane_of"][bad] == 1 and mix["rerun_in_dense_pool"] == 1
    assert all(f[0] == bad for f in mix["flagged"])
    assert mix["step_latency_ms"]["n"] == sum(r["steps"] - 1 for r in reqs)
    for k, r in enumerate(reqs):
        solo = srv.run([r], keep_results=True)
        assert solo["failed"] == 0
        x0, v0 = mix["results"][k]
        x1, v1 = solo["results"][0]
        assert torch.equal(x0, x1) and torch.equal(v0, v1), f"request {k}"
