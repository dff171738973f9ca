#!/usr/bin/env python3
"""Benchmark of the VBC hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--f 4] [--no-sweep] [--no-cpu]
                    [--no-paper-table] [--no-melt] [--no-serve] [--serve-requests 256]

Workload (default): N = 1,000,000 particles, cubic periodic box at number density 0.5,
uniform random start, standard VBC(1.5, 2.0, 0) on the polynomial soft core (E_r = 20,
r_r = 1, r_a = 1.5), well depth 5 kT, valency 4, list buffer 0.4; FP32 pair arithmetic
with FP64 counts, switching, integration and reductions; Langevin (BAOAB) kT = 1,
gamma = 0.1, dt = 0.005.  A step is one whole timestep of the hot path: list rebuild when
due, count pass, sparse dU/dn pass, force pass with the fused integrator update.

Prints ONE JSON line.  `value` is pair evaluations per second (ordered pairs inside the
interaction cutoff handled per step, times steps per second); timesteps/s is reported
beside it.  `roofline` is the dominant kernel's algorithmic bytes per launch over its
mean duration, timed with HIP events on the launch stream inside the timed region.
`serving` is the request stream: 256 independent simulations (N log-uniform in
[10^3, 2x10^5], valency 1..6, well depth 2..10 kT, density 0.3, 1000 Langevin steps each)
arriving as a Poisson stream at 0.8x the measured batched capacity, served by continuous
batching in one replica pool (2 GiB HBM budget, 64 replica slots, 2^21 particles) and,
on the same arrivals, one at a time; per-step latency percentiles come from device time
stamps written at the end of every step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "VBC pair evals/s + timesteps/s at N=1M (frac. HBM roofline); p99 step latency batched"
HBM_PEAK_GBS = 8000.0


def kernel_bytes(kind: str, N: int, kbar: float, precision: str, ntypes: int = 1) -> float:
    """Algorithmic HBM bytes of one launch of a kernel class, for the chosen layout.

    Every datum a launch needs is counted once: list entries are 2 bytes, counts per
    particle 2 bytes, positions/velocities/reference positions FP64 SoA, the type (4 bytes)
    only with several types; halo copies staged by several workgroups are cache re-reads,
    not algorithmic traffic."""
    sa = 8 if precision == "fp32" else 16
    ty = 4 if ntypes > 1 else 0
    if kind == "count":
        # list + nn + x (+ type)  ->  n (FP64) + (s, A)
        return N * (2 * kbar + 2 + 24 + ty + 8 + sa)
    if kind == "force":
        # list + nn + x (+ type) + (s, A) + tag + v (r/w) + x_next (w) + x_ref (r)
        return N * (2 * kbar + 2 + 24 + ty + sa + 4 + 48 + 24 + 24)
    if kind == "build":
        # x, v, tag, type read and gathered, cell tables, list written
        return N * (48 + 8 + 4 * 6 + 48 + 8 + 24 + 2 * kbar + 2)
    return float("nan")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary of this workload,
    or None if the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_fluid_N1000000_rho0.5_f4.json")
    src = os.path.join(ROOT, "paper_2609_07842_amd", "csrc", "vbc_kernels.hip")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != cur or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel]["traffic_bytes"]


def cpu_baseline(wl, target_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: full VBC forces of m
    particles of the N = 10^6 configuration (each needs O(N) scans for its own and its
    neighbours' counts).  Returns pair evaluations delivered per second."""
    import oracle
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(123)
    rc = max(wl.params["r_r"], wl.params["r_a"], wl.params["r_h"])
    tree = cKDTree(wl.x, boxsize=wl.L)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate on one batch of `cores` particles, then size the measured sample
    idx = rng.choice(wl.N, size=cores, replace=False)
    t0 = time.perf_counter()
    oracle.evaluate_subset(wl.x, wl.L, wl.params, idx)
    t_cal = time.perf_counter() - t0
    m = int(max(cores, min(4096, cores * max(1, round(target_s / max(t_cal, 1e-3))))))
    idx = rng.choice(wl.N, size=m, replace=False)
    t0 = time.perf_counter()
    oracle.evaluate_subset(wl.x, wl.L, wl.params, idx)
    dt = time.perf_counter() - t0
    pairs = sum(len(v) - 1 for v in tree.query_ball_point(wl.x[idx], rc))
    return {"value": pairs / dt, "unit": "pair evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} particles of the N={wl.N} start configuration: FP64 forces by the "
                      f"O(N^2) oracle ({pairs} pair evaluations in {dt:.1f} s)",
            "seconds": dt}


def achievable_copy(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy bandwidth (read + write bytes per second) of torch's copy
    kernel on 1 GiB buffers: the achievable HBM rate beside the nominal peak."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    a.copy_(b)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        a.copy_(b)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def measure_clusters(s, wl, torch, kbar, reps=5):
    """Cluster analysis of the bond graph on the state the timed steps left: one warm call,
    then `reps` calls between HIP events on the launch stream.  Algorithmic bytes per
    particle: two list sweeps (2 B per entry + 2 B count, own FP64 position, each), the
    type, five int32 scratch arrays written by the init pass, bonds written and read, the
    union-find parent written, read twice and written again, the per-root atomics (size,
    bond ends, smallest tag), and the label pass (parent, smallest tag, tag, label)."""
    s.clusters(hist_len=4096)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        lab, stats, hist = s.clusters(hist_len=4096)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    st = stats.cpu().numpy()[0]
    per_particle = 2 * (2 * kbar + 2 + 24) + 4 + 5 * 4 + 2 * 4 + 4 * 4 + 3 * 4 + 4 * 4
    nbytes = per_particle * wl.N
    return {"ms": ms, "clusters": int(st[0]), "P_inf": float(st[1]) / wl.N, "x_cyc": float(st[2]) / wl.N,
            "bonds_per_particle": float(st[3]) / wl.N, "bytes_model": nbytes,
            "achieved_GBs": nbytes / (ms * 1e-3) / 1e9,
            "timing": "HIP events around 5 calls of vbc_clusters (scratch init, hooking, counting, "
                      "labels and histograms) on the launch stream"}


def run_one(W, vbc, torch, f, steps, warmup, seed, profile=True, rho_max=0.0):
    from paper_2609_07842_amd import tune
    wl = W.headline(f=f, seed=seed)
    # brick edge and workgroup size from the autotuner's cache when it has this workload
    layout = tune.lookup(tune.fluid_key(wl.N, 0.5, "fp32")) or {}
    if rho_max:
        layout = dict(layout, rho_max=rho_max)
    print(f"[bench] device {tune._device_name()}: tuned layout {layout or 'none (automatic)'}",
          file=sys.stderr, flush=True)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, skin=W.SKIN), precision="fp32", **layout)
    s.set_state(wl.x, wl.v)
    integ = dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=seed)
    # warmup: relax the random start and reach a steady rebuild rate
    done = 0
    while done < warmup:
        k = min(500, warmup - done)
        s.step(k, **integ)
        done += k
    s.check()
    st0 = s.stats()[0]
    # timed region: K whole steps, launched as captured step graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, **integ)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.check()
    st1 = s.stats()[0]
    elapsed = t1 - t0
    evals = st1["evals"] - st0["evals"]
    pair_evals = (st1["pair_evals"] - st0["pair_evals"]) / max(evals, 1)
    builds = st1["builds"] - st0["builds"]
    kbar = st1["list_entries"] / wl.N
    prof, elapsed_prof = None, None
    if profile:
        # second timed region of K steps continuing the same trajectory, every kernel
        # launched individually between HIP events on the launch stream
        s.profile(True, max_launches=steps + 8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.step(steps, **integ)
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - t2
        prof = s.profile_read()
        s.profile(False)
        s.check()
    clusters = measure_clusters(s, wl, torch, kbar) if profile else None
    out = dict(wl=wl, elapsed=elapsed, pair_evals_per_step=pair_evals, builds=builds, kbar=kbar,
               prof=prof, elapsed_prof=elapsed_prof, opts=s.options(), clusters=clusters)
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def run_melt(W, vbc, torch, steps, warmup, seed):
    """Bead-spring melt: 20,000 chains x 50 beads (N = 10^6) at density 0.85, harmonic
    bonds k = 100, r0 = 1, every fifth bead a valency-1 sticker (well depth 8) counting only
    stickers, FP32 pair arithmetic, Langevin kT = 1.  The random-walk start packs beads at
    bond distance and overlapping chains, so the first `warmup` steps run in a layout sized
    for local densities up to 2 with a long list (k_max 256); the timed handle is then laid
    out for the relaxed melt (bricks of 3^3 cells keep the dense staging within LDS)."""
    wl = W.polymer_melt(seed=seed)
    integ = dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=seed)

    def make(**opts):
        return vbc.System(vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=50,
                                      k_bond=wl.k_bond, r0_bond=wl.r0, skin=W.SKIN),
                          precision="fp32", brick=3, **opts)
    s = make(k_max=256, rho_max=2.0)
    s.set_state(wl.x, wl.v, types=wl.types)
    s.step(warmup, **integ)
    s.check()
    x, v = (t.contiguous() for t in s.get_state())
    s.close()
    del s
    s = make()
    s.set_state(x, v, types=wl.types)
    s.step(200, **integ)
    s.check()
    st0 = s.stats()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps, **integ)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.check()
    st1 = s.stats()[0]
    pe = (st1["pair_evals"] - st0["pair_evals"]) / max(st1["evals"] - st0["evals"], 1)
    tsps = steps / dt
    return {"workload": "20,000 chains x 50 beads, density 0.85, bonds k=100 r0=1, stickers every "
                        "5th bead (f=1, eps=8kT, count stickers only), FP32 pair / FP64 integration, "
                        "Langevin kT=1 gamma=0.1 dt=0.005",
            "N": wl.N, "steps": steps, "timesteps_per_s": tsps, "pair_evals_per_s": tsps * pe,
            "pair_evals_per_step": pe, "list_entries_per_particle": st1["list_entries"] / wl.N,
            "steps_per_rebuild": steps / max(st1["builds"] - st0["builds"], 1),
            "layout": s.options()}


def run_paper_table(W, vbc, torch, steps=20000, warmup=2000, seed=8):
    """The configuration of the paper's cost table (Section 5, Table 1): N = 10^4 at density
    0.05, standard VBC(1.5, 2.0, 0), list buffer 0.4, valency 1..6; here well depth 5 kT,
    Langevin kT = 1, FP32 pair arithmetic.  Reported as seconds per 10^6 steps, the unit of
    the paper's table (its numbers are on an A100 with another neighbour-list backend:
    context, not a baseline)."""
    out = {}
    for f in (1, 2, 3, 4, 5, 6):
        wl = W.fluid(10_000, 0.05, float(f), E_a=5.0, seed=seed)
        s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, skin=W.SKIN), precision="fp32")
        s.set_state(wl.x, wl.v)
        integ = dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=seed)
        s.step(warmup, **integ)
        s.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, **integ)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.check()
        out[str(f)] = {"seconds_per_1e6_steps": dt / steps * 1e6, "timesteps_per_s": steps / dt}
        s.close()
    v = [x["seconds_per_1e6_steps"] for x in out.values()]
    out["flatness_max_over_min"] = max(v) / min(v)
    out["paper_A100_seconds_per_1e6_steps"] = {"1": 119, "2": 122, "3": 117, "4": 122, "5": 123, "6": 124}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--f", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-melt", action="store_true")
    ap.add_argument("--no-paper-table", action="store_true")
    ap.add_argument("--rho-max", type=float, default=0.0,
                    help="size the main run's layout for local densities up to this value")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one 512 MiB device-to-device copy (reference for byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus}, WORLD_SIZE={world} requested); "
              "this build runs each system on a single MI355X and has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_07842_amd import vbc
    from paper_2609_07842_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    main_run = run_one(W, vbc, torch, args.f, args.steps, args.warmup, args.seed, rho_max=args.rho_max)
    wl = main_run["wl"]
    K = args.steps
    tsps = K / main_run["elapsed"]
    pe_step = main_run["pair_evals_per_step"]
    prof = main_run["prof"]
    kernels = {k: {"mean_us": 1e3 * ms / n if n else None, "launches": n, "total_ms": ms}
               for k, (ms, n) in prof.items()}
    dom = max(("build", "count", "embed", "force"), key=lambda k: prof[k][0])
    ms, n = prof[dom]
    mean_s = ms / n / 1e3
    nbytes = kernel_bytes(dom, wl.N, main_run["kbar"], "fp32")
    achieved = nbytes / mean_s / 1e9
    copy_gbs = achievable_copy(torch)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "achievable_copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                "traffic": measured_traffic(dom),
                "bytes_per_launch": nbytes, "mean_launch_us": mean_s * 1e6,
                "timing": "HIP events around every launch in a second timed region of the same "
                          "K steps (individual launches instead of step graphs)",
                "ms_per_step_event_region": 1e3 * main_run["elapsed_prof"] / K}
    # whole-step view: all kernels' algorithmic bytes per step over the step time
    step_bytes = (kernel_bytes("count", wl.N, main_run["kbar"], "fp32")
                  + kernel_bytes("force", wl.N, main_run["kbar"], "fp32")
                  + kernel_bytes("build", wl.N, main_run["kbar"], "fp32") * main_run["builds"] / K)

    sweep = None
    if not args.no_sweep:
        # the same layout for every valency, sized for local densities up to 0.9: at f = 6
        # the fluid condenses within a few thousand steps and outgrows mean-density margins
        sweep = {"rho_max": 0.9}
        Ks = max(200, K // 2)
        for f in (1, 2, 3, 4, 5, 6):
            try:
                r = run_one(W, vbc, torch, float(f), Ks, max(500, args.warmup // 2), args.seed,
                            profile=False, rho_max=0.9)
            except vbc.VBCError as e:
                sweep[str(f)] = {"error": str(e)}
                continue
            ts = Ks / r["elapsed"]
            sweep[str(f)] = {"timesteps_per_s": ts, "pair_evals_per_s": ts * r["pair_evals_per_step"],
                             "builds": r["builds"], "steps_per_rebuild": Ks / max(r["builds"], 1),
                             "list_entries_per_particle": r["kbar"]}
        vals = [v["timesteps_per_s"] for k, v in sweep.items() if isinstance(v, dict) and "timesteps_per_s" in v]
        sweep["flatness_max_over_min"] = max(vals) / min(vals) if vals else None

    paper_table = None
    if not args.no_paper_table:
        print("[bench] paper cost-table configuration", file=sys.stderr, flush=True)
        paper_table = run_paper_table(W, vbc, torch)

    melt = None
    if not args.no_melt:
        print("[bench] polymer melt", file=sys.stderr, flush=True)
        melt = run_melt(W, vbc, torch, steps=1000, warmup=1000, seed=4)
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serve:
        from paper_2609_07842_amd import serve
        main_run.pop("system", None)
        torch.cuda.empty_cache()
        res = serve.serving_benchmark(n=args.serve_requests,
                                      log=lambda m: print(m, file=sys.stderr, flush=True))
        serving = {"p99_step_latency_ms_batched": res["batched"]["step_latency_ms"]["p99"],
                   "p50_step_latency_ms_batched": res["batched"]["step_latency_ms"]["p50"],
                   "p99_step_latency_ms_one_at_a_time": res["one_at_a_time"]["step_latency_ms"]["p99"],
                   "p50_step_latency_ms_one_at_a_time": res["one_at_a_time"]["step_latency_ms"]["p50"],
                   "throughput_batched_over_one_at_a_time": res["speedup_throughput"],
                   **res}

    cpu = None if args.no_cpu else cpu_baseline(wl)

    line = {
        "metric": METRIC,
        "value": tsps * pe_step,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * main_run["elapsed"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 counts/switching/integration/reductions",
        "data": "synthetic",
        "config": {"workload": "N=1,000,000 uniform-random start, density 0.5, valency 4, "
                               "eps=5kT, standard VBC(1.5,2.0,0), skin 0.4, Langevin kT=1 "
                               "gamma=0.1 dt=0.005",
                   "N": wl.N, "rho": 0.5, "f": args.f, "E_a": 5.0, "precision": "fp32_mixed",
                   "parallelism": "single GPU"},
        "timesteps_per_s": tsps,
        "particle_steps_per_s": tsps * wl.N,
        "pair_evals_per_step": pe_step,
        "list_entries_per_particle": main_run["kbar"],
        "steps_per_rebuild": K / max(main_run["builds"], 1),
        "layout": main_run["opts"],
        "kernels": kernels,
        "step_model_GBs": step_bytes * tsps / 1e9,
        "roofline": roofline,
        "cluster_analysis": main_run["clusters"],
        "f_sweep": sweep,
        "paper_table_config": paper_table,
        "polymer_melt": melt,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.calib_copy:
        # reference traffic for the byte counters: 512 MiB read + 512 MiB written by HIP's
        # own device-to-device copy kernel, then by torch's copy kernel
        import ctypes
        hip = ctypes.CDLL("libamdhip64.so")
        a = torch.empty(64 * 2**20, dtype=torch.int64, device="cuda")
        b = torch.ones_like(a)
        torch.cuda.synchronize()
        hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_int, ctypes.c_void_p]
        rc = hip.hipMemcpyAsync(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                a.numel() * 8, 3, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": a.numel() * 8, "hipMemcpyAsync_rc": rc}), file=sys.stderr)


if __name__ == "__main__":
    main()
