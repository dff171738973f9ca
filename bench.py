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
mean duration, timed with HIP events that the kernels' own dispatches record
(hipExtLaunchKernel) on the launch stream, in a region of the timed trajectory.
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


def _oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def _pairs_within(x, L, rc):
    """Ordered pairs closer than rc (the pair evaluations one VBC evaluation delivers)."""
    from scipy.spatial import cKDTree
    return 2 * len(cKDTree(x, boxsize=L).query_pairs(rc))


def cpu_baseline(wl, target_s=12.0):
    """The FP64 oracle on a bounded sample of the headline workload: full VBC forces of m
    particles of the N = 10^6 configuration (each needs O(N) scans for its own and its
    neighbours' counts).  Returns pair evaluations delivered per second."""
    import oracle
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(123)
    rc = max(wl.params["r_r"], wl.params["r_a"], wl.params["r_h"])
    tree = cKDTree(wl.x, boxsize=wl.L)
    cores = _oracle_threads()
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


_SMALL_CASE = """
import json, sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_2609_07842_amd import workloads as W
wl = W.small_fluid()
t0 = time.perf_counter(); oracle.evaluate(wl.x, wl.L, wl.params); t1 = time.perf_counter()
oracle.run(wl.x, wl.v, wl.L, wl.params, 100, kind=oracle.NVE, dt=0.005); t2 = time.perf_counter()
print(json.dumps({{"eval_s": t1 - t0, "run100_s": t2 - t1}}))
"""


def cpu_cases():
    """The oracle on the small cases beside the GPU: the N = 1000 NVE configuration in full
    (one evaluation and 100 velocity-Verlet steps, FP64) on all host threads and on one, and
    single evaluations of uniform fluids (density 0.3, f = 2) at N = 10^3 and 10^4 in full
    and at N = 10^5 as a sample of particles, with the full O(N^2) evaluation extrapolated
    from the N = 10^4 rate (labelled).  Pair visits are the three all-pairs sweeps over
    N (N - 1) ordered pairs of one evaluation; pair evaluations are the ordered pairs
    inside the cutoff."""
    import subprocess

    import oracle
    from paper_2609_07842_amd import workloads as W

    cores = _oracle_threads()
    out = {"cores": cores, "kind": "oracle"}
    wl = W.small_fluid()
    pe = _pairs_within(wl.x, wl.L, 2.0)
    t0 = time.perf_counter()
    oracle.evaluate(wl.x, wl.L, wl.params)
    t1 = time.perf_counter()
    oracle.run(wl.x, wl.v, wl.L, wl.params, 100, kind=oracle.NVE, dt=0.005)
    t2 = time.perf_counter()
    visits = 3 * wl.N * (wl.N - 1)
    out["small_fluid_N1000_nve100"] = {
        "eval_s": t1 - t0, "run100_s": t2 - t1, "steps_per_s": 100 / (t2 - t1),
        "particle_steps_per_s": 100 * wl.N / (t2 - t1), "pair_visits_per_s": 101 * visits / (t2 - t0),
        "pair_evals_per_eval": pe}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _SMALL_CASE.format(root=ROOT)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode == 0:
        one = json.loads(r.stdout.strip().splitlines()[-1])
        one["steps_per_s"] = 100 / one["run100_s"]
        one["particle_steps_per_s"] = 100 * wl.N / one["run100_s"]
        out["small_fluid_N1000_nve100_one_core"] = one
    else:
        out["small_fluid_N1000_nve100_one_core"] = {"error": r.stderr[-400:]}
    rate_1e4 = None
    for N in (1_000, 10_000):
        f = W.fluid(N, 0.3, 2.0, E_a=5.0, seed=1)
        t0 = time.perf_counter()
        oracle.evaluate(f.x, f.L, f.params)
        dt = time.perf_counter() - t0
        v = 3 * N * (N - 1)
        out[f"eval_N{N}"] = {"seconds": dt, "pair_visits_per_s": v / dt,
                             "pair_evals_per_s": _pairs_within(f.x, f.L, 2.0) / dt}
        rate_1e4 = v / dt
    N = 100_000
    f = W.fluid(N, 0.3, 2.0, E_a=5.0, seed=1)
    idx = np.random.default_rng(7).choice(N, size=max(cores, 64), replace=False)
    t0 = time.perf_counter()
    oracle.evaluate_subset(f.x, f.L, f.params, idx)
    dt = time.perf_counter() - t0
    out["eval_N100000"] = {"sample_particles": len(idx), "sample_seconds": dt,
                           "full_eval_seconds_extrapolated_N2_from_N1e4": 3 * N * (N - 1) / rate_1e4,
                           "note": "full O(N^2) evaluation not run: time extrapolated as N^2 from the "
                                   "measured N = 10^4 pair-visit rate"}
    return out


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


RELAX_STEPS = 2000


def run_one(W, vbc, torch, f, steps, warmup, seed, profile=True, rho_max=0.0, relax=RELAX_STEPS):
    from paper_2609_07842_amd import tune
    wl = W.headline(f=f, seed=seed)
    # brick edge and workgroup size from the autotuner's cache when it has this workload
    key = tune.fluid_key(wl.N, 0.5, "fp32")
    layout = tune.lookup(key) or {}
    why = tune.stale(key)
    if rho_max:
        layout = dict(layout, rho_max=rho_max)
    print(f"[bench] device {tune._device_name()}: tuned layout "
          f"{layout or 'none (automatic)'}{'' if why is None else ' (tuned cache not used: ' + why + ')'}",
          file=sys.stderr, flush=True)
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params, skin=W.SKIN), precision="fp32", **layout)
    s.set_state(wl.x, wl.v)
    integ = dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=seed)
    # input preparation (untimed): relax the uniform random start, so that the steps timed
    # run at the fluid's steady list-rebuild rate rather than in its first transient; then
    # the warm-up steps
    for n in [500] * (relax // 500) + [relax % 500] + [500] * (warmup // 500) + [warmup % 500]:
        if n:
            s.step(n, **integ)
    s.check()
    # capture the step graphs of the timed call before the timed region
    s.prepare_step(steps, **integ)
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
    thermo = prof = elapsed_prof = builds_prof = None
    if profile:
        # K more steps with the energy and the virial of every step accumulated (pass 2 in
        # full: forces, energy, virial), timed the same way
        s.thermo(True)
        s.prepare_step(steps, **integ)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.step(steps, **integ)
        torch.cuda.synchronize()
        el = time.perf_counter() - t2
        th = s.thermo_read()[0]
        s.thermo(False)
        s.check()
        thermo = {"timesteps_per_s": steps / el, "ms_per_step": 1e3 * el / steps,
                  "steps_accumulated": th["steps"], "mean_U_per_particle": th["sum"][0] / max(th["steps"], 1) / wl.N,
                  "mean_W_per_particle": th["sum"][1] / max(th["steps"], 1) / wl.N,
                  "what": "every step also sums the pair energies and the virial (scalar and "
                          "tensor) per brick in FP64 and reduces them per replica"}
        # a third region of K steps continuing the same trajectory, every kernel launched
        # individually, its dispatch recording a pair of HIP events on the launch stream
        s.profile(True, max_launches=steps + 8)
        st2 = s.stats()[0]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        s.step(steps, **integ)
        torch.cuda.synchronize()
        elapsed_prof = time.perf_counter() - t2
        prof = s.profile_read()
        s.profile(False)
        s.check()
        builds_prof = s.stats()[0]["builds"] - st2["builds"]
    clusters = measure_clusters(s, wl, torch, kbar) if profile else None
    out = dict(wl=wl, elapsed=elapsed, pair_evals_per_step=pair_evals, builds=builds, kbar=kbar,
               prof=prof, elapsed_prof=elapsed_prof, builds_prof=builds_prof, thermo=thermo,
               opts=s.options(), clusters=clusters, relax=relax)
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def kernel_table(main_run, N, steps):
    """Per kernel class: time per launch and per step from the event-timed region, and its
    algorithmic bytes over that time as a fraction of HBM peak.  The list-build class
    launches on every step but builds only when a particle has moved more than half the
    buffer, so its bytes are those of one build and its time is the class total over the
    builds that happened (empty launches included)."""
    prof, kbar = main_run["prof"], main_run["kbar"]
    out = {}
    for k in ("build", "count", "embed", "force", "kick", "reduce"):
        ms, n = prof[k]
        e = {"launches": n, "total_ms": ms, "per_step_us": 1e3 * ms / steps,
             "mean_launch_us": 1e3 * ms / n if n else None}
        nb = kernel_bytes(k, N, kbar, "fp32")
        if k == "build":
            nbld = main_run["builds_prof"] or 0
            e["builds"] = nbld
            e["us_per_build"] = 1e3 * ms / nbld if nbld else None
            t_unit = ms / nbld * 1e-3 if nbld else None
        else:
            t_unit = ms / n * 1e-3 if n else None
        if t_unit and nb == nb:
            e["bytes_per_unit"] = nb
            e["achieved_GBs"] = nb / t_unit / 1e9
            e["frac"] = e["achieved_GBs"] / HBM_PEAK_GBS
            e["traffic"] = measured_traffic(k)
        out[k] = e
    return out


def run_melt(W, vbc, torch, steps, warmup, seed):
    """Bead-spring melt: 20,000 chains x 50 beads (N = 10^6) at density 0.85, harmonic
    bonds k = 100, r0 = 1, every fifth bead a valency-1 sticker (well depth 8) counting only
    stickers, FP32 pair arithmetic, Langevin kT = 1.  The random-walk start packs beads at
    bond distance and overlapping chains, so the first `warmup` steps run in a layout sized
    for local densities up to 2 with a long list (k_max 256); the timed handle is then laid
    out for the relaxed melt, with the brick and workgroup size the autotuner cached for it
    (bricks of 3^3 cells, the default, keep the dense staging within LDS)."""
    from paper_2609_07842_amd import tune
    wl, x, v = tune.relaxed_melt(seed=seed, warmup=warmup)
    integ = tune.melt_integrator(wl)
    key = tune.melt_key("fp32")
    lay = tune.lookup(key)
    if lay is None:
        print(f"[bench] melt: default layout (autotune cache: {tune.stale(key)})", file=sys.stderr, flush=True)
        lay = dict(brick=3)
    else:
        print(f"[bench] melt: tuned layout {lay}", file=sys.stderr, flush=True)
    s = tune.melt_system(wl, "fp32", **lay)
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


def gpu_cases(W, vbc, torch):
    """The GPU on the oracle's small cases: the N = 1000 NVE configuration in full (FP64:
    one force evaluation, then 100 velocity-Verlet steps) and single force evaluations of
    uniform fluids (density 0.3, f = 2) at N = 10^3, 10^4 and 10^5 in both precisions (mean
    of 20 evaluations after one warm call, energies and virial included)."""
    out = {}
    wl = W.small_fluid()
    s = vbc.System(vbc.replica(wl.N, wl.L, wl.params), precision="fp64")
    s.set_state(wl.x, wl.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.force()
    s.step(100, integrator="nve", dt=0.005)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.check()
    s.close()
    out["small_fluid_N1000_nve100"] = {"seconds": dt, "steps_per_s": 100 / dt,
                                       "note": "wall time of the first evaluation (list build "
                                               "included) and 100 steps (graph capture included)"}
    for N in (1_000, 10_000, 100_000):
        f = W.fluid(N, 0.3, 2.0, E_a=5.0, seed=1)
        for prec in ("fp64", "fp32"):
            s = vbc.System(vbc.replica(N, f.L, f.params), precision=prec)
            s.set_state(f.x)
            s.force()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(20):
                s.force()
            ev1.record()
            torch.cuda.synchronize()
            s.check()
            out[f"eval_N{N}_{prec}"] = {"ms_per_eval": ev0.elapsed_time(ev1) / 20}
            s.close()
    torch.cuda.empty_cache()
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
    ap.add_argument("--no-small", action="store_true", help="skip the small GPU cases beside the oracle's")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-melt", action="store_true")
    ap.add_argument("--no-paper-table", action="store_true")
    ap.add_argument("--relax", type=int, default=RELAX_STEPS,
                    help="untimed Langevin steps that relax the random start before the warm-up")
    ap.add_argument("--rho-max", type=float, default=0.0,
                    help="size the main run's layout for local densities up to this value")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one 512 MiB device-to-device copy (reference for byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus}, WORLD_SIZE={world} requested); "
              "the library runs each system on a single MI355X and has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_07842_amd import vbc
    from paper_2609_07842_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    main_run = run_one(W, vbc, torch, args.f, args.steps, args.warmup, args.seed, rho_max=args.rho_max,
                       relax=args.relax)
    wl = main_run["wl"]
    K = args.steps
    tsps = K / main_run["elapsed"]
    pe_step = main_run["pair_evals_per_step"]
    kernels = kernel_table(main_run, wl.N, K)
    # the dominant kernel: the largest share of the step time
    dom = max(("build", "count", "embed", "force"), key=lambda k: kernels[k]["per_step_us"])
    kd = kernels[dom]
    copy_gbs = achievable_copy(torch)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kd.get("achieved_GBs"), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": kd.get("frac"), "traffic": kd.get("traffic"),
                "bytes_per_launch": kd.get("bytes_per_unit"),
                "mean_launch_us": kd["us_per_build"] if dom == "build" else kd["mean_launch_us"],
                "achievable_copy_GBs": copy_gbs,
                "frac_of_copy": kd["achieved_GBs"] / copy_gbs if kd.get("achieved_GBs") else None,
                "per_kernel_frac": {k: v.get("frac") for k, v in kernels.items() if v.get("frac")},
                "timing": "HIP events recorded by each kernel class's own dispatches "
                          "(hipExtLaunchKernel: start of its first kernel, end of its last) on the "
                          "launch stream, in a third region of K steps (individual launches instead "
                          "of step graphs); the list build's bytes are one build's, over its time "
                          "per build",
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
                             "list_entries_per_particle": r["kbar"],
                             # step time per list entry: separates the longer lists of a
                             # condensing fluid from the cost of the kernels themselves
                             "ps_per_list_entry": 1e12 / ts / (r["wl"].N * r["kbar"])}
        rows = [v for k, v in sweep.items() if isinstance(v, dict) and "timesteps_per_s" in v]
        vals = [v["timesteps_per_s"] for v in rows]
        sweep["flatness_max_over_min"] = max(vals) / min(vals) if vals else None
        per = [v["ps_per_list_entry"] for v in rows]
        sweep["flatness_per_list_entry_max_over_min"] = max(per) / min(per) if per else None

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

    gpu_small = None if args.no_small else gpu_cases(W, vbc, torch)
    cpu = None
    if not args.no_cpu:
        print("[bench] oracle on the host", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl)
        cpu["cases"] = cpu_cases()

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
        "config": {"workload": "N=1,000,000 fluid at density 0.5, valency 4, eps=5kT, standard "
                               "VBC(1.5,2.0,0), skin 0.4, Langevin kT=1 gamma=0.1 dt=0.005; "
                               f"uniform-random start relaxed by {main_run['relax']} untimed steps "
                               "before the warm-up",
                   "N": wl.N, "rho": 0.5, "f": args.f, "E_a": 5.0, "precision": "fp32_mixed",
                   "parallelism": "single GPU"},
        "timesteps_per_s": tsps,
        "timesteps_per_s_with_energy_virial": (main_run["thermo"] or {}).get("timesteps_per_s"),
        "energy_virial_run": main_run["thermo"],
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
        "gpu_small_cases": gpu_small,
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
