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
    assert mix["flagged"] == []
    assert mix["mean_live"] > 1.5                     # requests really ran together
    assert mix["queue_wait_s"]["p99"] > 0.0           # and admission made some wait
    assert mix["step_latency_ms"]["n"] == sum(q["steps"] - 1 for q in reqs)
    for k, q in enumerate(reqs):
        solo = srv.run([q], keep_results=True)
        x0, v0 = mix["results"][k]
        x1, v1 = solo["results"][0]
        assert torch.equal(x0, x1) and torch.equal(v0, v1), f"request {k}"
