"""Continuous-batching request loop over a replica pool (libvbc's vbc_pool_* calls).

Each request is an independent simulation (its own size, valency, well depth, noise
seed and step count).  Requests wait in a FIFO queue until a replica slot, enough
particle indices and enough of the HBM budget are free (admission by workspace
footprint, vbc_replica_footprint); admitted requests run together, as one pool, one
captured step graph of `steps_per_tick` steps per launch; a request that has done its
steps has its final state copied out and leaves, and queued requests take its place
between two launches while the others keep running.

Everything numeric runs in the library's kernels; this module only decides admission
and ordering, and reads device time stamps (one per step, vbc_stamps) and HIP events
for the latency figures.  The same loop with at most one live replica is the
one-at-a-time baseline.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import vbc as _vbc
from . import workloads as W


@dataclass
class ServerConfig:
    budget_bytes: int = 2 << 30      # HBM the live replicas of the main pool may occupy
    max_replicas: int = 64
    max_particles: int = 1 << 21
    precision: str = "fp32"
    steps_per_tick: int = 8
    rho_max: float = 0.3             # densest request the main pool is laid out for
    # a request whose local density outgrows the main pool's layout (it condenses), or that
    # trips any other error flag, is evicted and run again from its initial state in a
    # second pool laid out for local densities up to dense_rho_max
    dense_rho_max: float = 1.0
    dense_budget_bytes: int = 1 << 30
    dense_max_replicas: int = 16
    dense_max_particles: int = 1 << 19
    max_attempts: int = 2            # attempts per request (main pool, then dense pool)
    check_every: int = 16            # ticks between reads of the running requests' flags
    n_range: tuple = (1_000, 200_000)
    skin: float = 0.4
    integrator: dict = field(default_factory=lambda: dict(integrator="langevin", dt=0.005,
                                                          kT=1.0, gamma=0.1, seed=2024))
    max_inflight: int = 6            # step launches the host may run ahead of the GPU
    max_active: int = 0              # 0 = no limit beyond the pools; 1 = one at a time
    brick: int = 0                   # 0 = the tuned choice if cached, else the library's
    block: int = 0


def request_desc(req, skin=0.4):
    """Replica description of a request dict (N, f, E_a, rho, seed)."""
    L = W.box_length(req["N"], req["rho"])
    return _vbc.replica(req["N"], L, W.vbc_params(E_a=req["E_a"], f=req["f"]), skin=skin,
                        seed=req["seed"])


def layout_for(cfg: ServerConfig, rho_max=None):
    """List length and staging capacity that cover every request size at the design
    density (the largest automatic choice over a log grid of sizes), the range of
    slots-per-brick such requests need, and the smallest workspace bytes per slot."""
    rho = cfg.rho_max if rho_max is None else rho_max
    k_max = stage_cap = bcap_max = 0
    bcap_min = 1 << 30
    # a log grid of sizes, plus the sizes just below each change of the cell count per
    # axis (there the cells are largest and hold the most particles)
    p = W.vbc_params()
    rl = max(p["r_r"], p["r_a"], p["r_h"]) + cfg.skin
    worst = [math.floor(cfg.rho_max * ((nc + 1) * rl) ** 3 * (1 - 1e-6)) for nc in range(3, 1024)]
    grid = np.concatenate([np.rint(np.geomspace(cfg.n_range[0], cfg.n_range[1], 64)),
                           [n for n in worst if cfg.n_range[0] <= n <= cfg.n_range[1]]])
    grid = np.unique(grid.astype(int))
    descs = [request_desc(dict(N=int(N), f=1.0, E_a=5.0, rho=cfg.rho_max, seed=0), cfg.skin)
             for N in grid]
    extra = dict(rho_max=rho) if rho > cfg.rho_max else {}
    for d in descs:
        fp = _vbc.footprint(d, cfg.precision, brick=cfg.brick, **extra)
        k_max, stage_cap = max(k_max, fp["k_max"]), max(stage_cap, fp["stage_cap"])
        bcap_max, bcap_min = max(bcap_max, fp["bcap"]), min(bcap_min, fp["bcap"])
    per_slot = min(fp["bytes"] / fp["slots"] for fp in
                   (_vbc.footprint(d, cfg.precision, k_max=k_max, stage_cap=stage_cap, brick=cfg.brick, **extra)
                    for d in descs))
    return dict(k_max=k_max, stage_cap=stage_cap, bcap_max=bcap_max, bcap_min=bcap_min,
                bytes_per_slot=per_slot, rho_max=rho)


class Lane:
    """One replica pool of the server with its layout, capacity, occupancy and step
    stamps."""

    def __init__(self, srv, name, rho_max, budget, max_replicas, max_particles):
        c = srv.cfg
        self.name, self.cfg, self.torch = name, c, srv.torch
        lay = layout_for(c, rho_max)
        self.rho_max = rho_max
        self.k_max, self.stage_cap = lay["k_max"], lay["stage_cap"]
        self.budget, self.max_replicas, self.max_particles = budget, max_replicas, max_particles
        # capacities that the byte budget reaches first: a replica's slots cost at least
        # bytes_per_slot each, and its bricks hold at least bcap_min slots
        max_slots = int(budget / lay["bytes_per_slot"]) + 1
        max_bricks = max_slots // lay["bcap_min"] + max_replicas
        caps = dict(max_replicas=max_replicas, max_types=1, max_particles=max_particles,
                    max_slots=max(max_slots, max_particles), max_bricks=max_bricks,
                    max_cells=max_bricks * 64, max_bcap=max(lay["bcap_max"], 64), chains=False)
        self.pool = _vbc.Pool(caps, precision=c.precision, k_max=self.k_max, stage_cap=self.stage_cap,
                              brick=c.brick, block=c.block, rho_max=rho_max if rho_max > c.rho_max else 0.0,
                              device=srv.device)
        self.reset()

    def reset(self):
        self.active = {}      # slot -> [request index, ticks left, first step, flags seen]
        self.used_bytes = self.used_particles = 0
        self.gstep = 0
        self.stamps = []
        self.busy = set()     # first step of a tick preceded by admissions or a sync
        self.since_read = 0
        self.ticks_since_check = 0

    def footprint(self, req):
        extra = dict(rho_max=self.rho_max) if self.rho_max > self.cfg.rho_max else {}
        return _vbc.footprint(request_desc(req, self.cfg.skin), self.cfg.precision,
                              k_max=self.k_max, stage_cap=self.stage_cap, brick=self.cfg.brick,
                              **extra)["bytes"]

    def warm(self):
        """Capture the step graphs (both buffer parities) on a tiny replica."""
        c = self.cfg
        req = dict(N=c.n_range[0], f=2.0, E_a=5.0, rho=c.rho_max, seed=1)
        d = request_desc(req, c.skin)
        x = W.uniform_positions(req["N"], d["L"][0], 1)
        r = self.pool.admit(d, x)
        for n in (c.steps_per_tick, c.steps_per_tick + 1, c.steps_per_tick):
            self.pool.step(n, **c.integrator)
        self.pool.check()
        self.pool.retire(r)

    def drain_stamps(self):
        self.stamps.append(self.pool.stamps_read())
        self.since_read = 0


class Server:
    def __init__(self, cfg: ServerConfig | None = None, device="cuda"):
        import torch

        self.torch = torch
        self.cfg = cfg or ServerConfig()
        c = self.cfg
        if not c.brick and not c.block:
            from . import tune
            best = tune.lookup(tune.pool_key(c))
            if best:
                c.brick, c.block = best["brick"], best["block"]
        self.device = torch.device(device) if isinstance(device, str) else device
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.lanes = [Lane(self, "main", c.rho_max, c.budget_bytes, c.max_replicas, c.max_particles)]
        if c.max_attempts > 1:
            self.lanes.append(Lane(self, "dense", c.dense_rho_max, c.dense_budget_bytes,
                                   c.dense_max_replicas, c.dense_max_particles))
        self.pool = self.lanes[0].pool
        self.k_max, self.stage_cap = self.lanes[0].k_max, self.lanes[0].stage_cap
        self.stream = torch.cuda.current_stream(self.device)
        for ln in self.lanes:
            ln.warm()
        torch.cuda.synchronize(self.device)

    def footprint(self, req):
        return self.lanes[0].footprint(req)

    def run(self, requests, arrivals=None, keep_results=False):
        """Serve `requests` (dicts with N, f, E_a, rho, seed, steps and device tensors x, v
        of shape (N, 3)); arrivals[k] = seconds after the start at which request k
        arrives (None: all at once).  Returns per-request timings, per-step latencies and
        totals over the requests that completed without an error flag.

        The running requests' flags are read every `check_every` ticks and whenever one
        finishes (each read synchronises and clears the flags, so they are kept per request
        until it leaves).  A request with an error flag (list or staging overflow, a
        non-finite coordinate, a particle lost between list builds) is evicted at once and,
        while attempts are left, queued again from its initial state for the dense pool;
        otherwise it is marked failed.  Failed requests and evicted attempts count in no
        throughput or latency figure."""
        torch, cfg = self.torch, self.cfg
        S = cfg.steps_per_tick
        lanes = self.lanes
        n_req = len(requests)
        arr = np.zeros(n_req) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
        order = np.argsort(arr, kind="stable")
        fps = [[ln.footprint(q) for q in requests] for ln in lanes]
        for k, q in enumerate(requests):
            if q["steps"] % S:
                raise ValueError("request steps must be a multiple of steps_per_tick")
            if fps[0][k] > cfg.budget_bytes or q["N"] > cfg.max_particles:
                raise ValueError(f"request {k} can never fit the pool")
        for ln in lanes:
            ln.reset()
        ev_start = torch.cuda.Event(enable_timing=True)
        ticks = []                      # (event, lane index)
        queues = [deque() for _ in lanes]
        nxt = 0
        admit_t = np.full(n_req, np.nan)
        first_step = np.zeros(n_req, dtype=np.int64)
        lane_of = np.zeros(n_req, dtype=np.int64)
        attempts = np.zeros(n_req, dtype=np.int64)
        done_tick = np.full(n_req, -1, dtype=np.int64)
        failed = np.zeros(n_req, dtype=bool)
        final_flags = np.zeros(n_req, dtype=np.int64)  # flags of the run that completed
        results = [None] * n_req
        flagged = []                    # (request, lane, flags, what happened)

        def read_flags(li, finished):
            """Read lane li's flags, keep them per request, evict the requests with an
            error, and retire the finished ones."""
            ln = lanes[li]
            ln.busy.add(ln.gstep)
            st, flags = ln.pool.check(raise_on_error=False)
            for r, a in ln.active.items():
                a[3] |= flags[r] & ~_vbc.FLAG_REBUILD
            for r in list(ln.active):
                k, left, g0, fl = ln.active[r]
                if fl:
                    what = "failed"
                    if attempts[k] < cfg.max_attempts and li + 1 < len(lanes):
                        what = f"evicted to the {lanes[li + 1].name} pool"
                        queues[li + 1].appendleft(k)
                        lane_of[k] = li + 1
                    else:
                        failed[k] = True
                    flagged.append((k, ln.name, int(fl), what))
                elif r in finished:
                    final_flags[k] = fl
                    if keep_results:
                        x, v = ln.pool.get_state(r)
                        results[k] = (x.clone(), v.clone())
                    done_tick[k] = len(ticks) - 1
                else:
                    continue
                ln.pool.retire(r)
                ln.used_bytes -= fps[li][k]
                ln.used_particles -= requests[k]["N"]
                del ln.active[r]
            ln.ticks_since_check = 0

        for ln in lanes:
            ln.pool.stamps(True)
        ev_start.record(self.stream)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        while nxt < n_req or any(queues) or any(ln.active for ln in lanes):
            now = time.perf_counter() - t0
            while nxt < n_req and arr[order[nxt]] <= now:
                queues[0].append(int(order[nxt]))
                nxt += 1
            # admission: FIFO per pool, while the head fits
            for li, ln in enumerate(lanes):
                q_ = queues[li]
                while q_:
                    k = q_[0]
                    q = requests[k]
                    if cfg.max_active and sum(len(x.active) for x in lanes) >= cfg.max_active:
                        break
                    if (len(ln.active) >= ln.max_replicas or ln.used_bytes + fps[li][k] > ln.budget
                            or ln.used_particles + q["N"] > ln.max_particles):
                        break
                    try:
                        r = ln.pool.admit(request_desc(q, cfg.skin), q["x"], q["v"])
                    except _vbc.VBCError as e:
                        if e.status != _vbc.VBC_ERR_CAPACITY:
                            raise
                        break  # no contiguous range now: wait for a retirement
                    q_.popleft()
                    attempts[k] += 1
                    ln.active[r] = [k, q["steps"] // S, ln.gstep, 0]
                    if np.isnan(admit_t[k]):
                        admit_t[k] = time.perf_counter() - t0
                    ln.busy.add(ln.gstep)
                    first_step[k] = ln.gstep
                    ln.used_bytes += fps[li][k]
                    ln.used_particles += q["N"]
            if not any(ln.active for ln in lanes):
                if nxt < n_req:
                    time.sleep(max(0.0, min(arr[order[nxt]] - (time.perf_counter() - t0), 0.01)))
                continue
            for li, ln in enumerate(lanes):
                if not ln.active:
                    continue
                ln.pool.step(S, **cfg.integrator)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.stream)
                ticks.append((ev, li))
                ln.gstep += S
                ln.since_read += S
                ln.ticks_since_check += 1
                finished = set()
                for r, a in ln.active.items():
                    a[1] -= 1
                    if a[1] == 0:
                        finished.add(r)
                if finished or ln.ticks_since_check >= cfg.check_every:
                    read_flags(li, finished)
                if ln.since_read > (1 << 15):
                    ln.drain_stamps()
            if len(ticks) > cfg.max_inflight:
                ticks[-cfg.max_inflight - 1][0].synchronize()
        for ln in lanes:
            ln.drain_stamps()
            ln.pool.stamps(False)
        torch.cuda.synchronize(self.device)
        t_tick = np.array([ev_start.elapsed_time(ev) * 1e-3 for ev, _ in ticks])
        lane_stamps = []
        for ln in lanes:
            st = np.concatenate(ln.stamps) if ln.stamps else np.zeros(0)
            if len(st) != ln.gstep:
                raise RuntimeError(f"{ln.name} pool: expected {ln.gstep} step stamps, got {len(st)}")
            lane_stamps.append(st)
        # per-step latency: interval between a request's successive step completions
        ok = [k for k in range(n_req) if not failed[k]]
        lat, quiet = [], []
        for k in ok:
            q, li, g0 = requests[k], lane_of[k], first_step[k]
            st = lane_stamps[li]
            busy = np.zeros(len(st) + 1, dtype=bool)
            for g in lanes[li].busy:
                if g < busy.size:
                    busy[g] = True
            d = np.diff(st[g0:g0 + q["steps"]])
            lat.append(d)
            quiet.append(d[~busy[g0 + 1:g0 + q["steps"]]])  # interval ending at step g0 + 1 + m
        lat = np.concatenate(lat) if lat else np.zeros(0)
        quiet = np.concatenate(quiet) if quiet else np.zeros(0)
        done = t_tick[done_tick[ok]] if ok else np.zeros(0)
        req_lat = done - arr[ok]
        makespan = float(t_tick.max()) if len(t_tick) else 0.0
        n_steps = sum(requests[k]["steps"] for k in ok)
        p_steps = sum(requests[k]["steps"] * requests[k]["N"] for k in ok)
        pct = lambda a, p: float(np.percentile(a, p)) if a.size else None
        return dict(
            makespan_s=makespan,
            requests_per_s=len(ok) / makespan if makespan else 0.0,
            request_steps_per_s=n_steps / makespan if makespan else 0.0,
            particle_steps_per_s=p_steps / makespan if makespan else 0.0,
            step_latency_ms=dict(p50=1e3 * pct(lat, 50), p99=1e3 * pct(lat, 99),
                                 mean=1e3 * float(lat.mean()), n=int(lat.size)),
            # the same over the steps whose tick did not start with admissions or a host sync
            step_latency_ms_between_events=dict(
                p50=1e3 * pct(quiet, 50) if quiet.size else None,
                p99=1e3 * pct(quiet, 99) if quiet.size else None,
                n=int(quiet.size)),
            request_latency_s=dict(p50=pct(req_lat, 50), p99=pct(req_lat, 99),
                                   max=float(req_lat.max()) if req_lat.size else None),
            queue_wait_s=dict(p50=float(np.nanpercentile(admit_t - arr, 50)),
                              p99=float(np.nanpercentile(admit_t - arr, 99))),
            global_steps=int(sum(ln.gstep for ln in lanes)),
            mean_live=float(sum(requests[k]["steps"] for k in range(n_req)) / max(lanes[0].gstep, 1)),
            completed=len(ok), failed=int(failed.sum()),
            # completed requests whose counted run raised an error flag (kept per request over
            # every flag read of its run): zero unless eviction failed to catch one
            flagged_in_figures=int(sum(1 for k in ok if final_flags[k])),
            rerun_in_dense_pool=int(sum(1 for k in ok if lane_of[k] > 0)),
            flagged=flagged,
            lane_of=lane_of.tolist(),
            results=results if keep_results else None,
        )


def make_requests(n=256, seed=5, rho=0.3, steps=1000, device="cuda", n_range=(1_000, 200_000)):
    """The request stream: sizes, valencies, well depths and noise seeds from the seeded
    generator, initial states (uniform positions, Maxwell-Boltzmann velocities at kT = 1)
    placed in device memory up front."""
    import torch

    reqs = W.serving_requests(n=n, seed=seed, rho=rho, N_min=n_range[0], N_max=n_range[1], steps=steps)
    for q in reqs:
        L = W.box_length(q["N"], rho)
        q["x"] = torch.from_numpy(W.uniform_positions(q["N"], L, q["seed"])).to(device)
        q["v"] = torch.from_numpy(W.maxwell_boltzmann(q["N"], 1.0, q["seed"] + 1)).to(device)
    return reqs


def poisson_arrivals(reqs, rate):
    """Arrival times (s) from the stream's unit-rate exponential gaps at `rate` per s."""
    return np.cumsum([q["gap"] for q in reqs]) / rate


def serving_benchmark(n=256, steps=1000, seed=5, load=0.8, cfg=None, log=None):
    """Capacity with every request queued at t = 0, then Poisson arrivals at `load` x that
    capacity served batched and one at a time (same arrivals, same pool)."""
    cfg = cfg or ServerConfig()
    say = log or (lambda *a: None)
    reqs = make_requests(n=n, seed=seed, rho=cfg.rho_max, steps=steps, n_range=cfg.n_range)
    srv = Server(cfg)
    say(f"[serve] pool: k_max {srv.k_max} stage_cap {srv.stage_cap} "
        f"workspace {srv.pool.ws_bytes / 2**30:.2f} GiB")
    sat = srv.run(reqs)
    say(f"[serve] saturated: {sat['requests_per_s']:.1f} req/s, mean live {sat['mean_live']:.1f}")
    rate = load * sat["requests_per_s"]
    arrivals = poisson_arrivals(reqs, rate)
    batched = srv.run(reqs, arrivals)
    say(f"[serve] batched at {rate:.1f} req/s: step p99 {batched['step_latency_ms']['p99']:.3f} ms")
    srv.cfg.max_active = 1
    single = srv.run(reqs, arrivals)
    srv.cfg.max_active = 0
    say(f"[serve] one at a time: {single['requests_per_s']:.1f} req/s")
    strip = lambda d: {k: v for k, v in d.items() if k not in ("results", "flagged", "lane_of")}
    return dict(requests=n, steps_per_request=steps, arrival_rate_per_s=rate, load=load,
                steps_per_tick=cfg.steps_per_tick, budget_bytes=cfg.budget_bytes,
                max_replicas=cfg.max_replicas, max_particles=cfg.max_particles,
                dense_pool=dict(rho_max=cfg.dense_rho_max, budget_bytes=cfg.dense_budget_bytes,
                                max_replicas=cfg.dense_max_replicas),
                mean_N=float(np.mean([q["N"] for q in reqs])),
                saturated=strip(sat), batched=strip(batched), one_at_a_time=strip(single),
                # requests counted in the figures although an error flag was raised for them:
                # none by construction (a flagged attempt is evicted, see Server.run)
                flagged=sum(r["flagged_in_figures"] for r in (sat, batched, single)),
                evictions=len(sat["flagged"]) + len(batched["flagged"]) + len(single["flagged"]),
                failed=sat["failed"] + batched["failed"] + single["failed"],
                flag_events=[dict(request=k, pool=p, flags=f, action=a)
                             for r in (sat, batched, single) for (k, p, f, a) in r["flagged"]][:32],
                speedup_throughput=batched["particle_steps_per_s"] / single["particle_steps_per_s"])


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="serve the synthetic request stream on one GPU")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--mode", choices=("all", "saturated"), default="all",
                    help="all: capacity, batched Poisson stream and one at a time; "
                         "saturated: every request queued at t = 0 only")
    a = ap.parse_args()
    say = lambda m: print(m, file=sys.stderr, flush=True)
    if a.mode == "all":
        res = serving_benchmark(n=a.requests, steps=a.steps, log=say)
    else:
        cfg = ServerConfig()
        reqs = make_requests(n=a.requests, rho=cfg.rho_max, steps=a.steps, n_range=cfg.n_range)
        res = Server(cfg).run(reqs)
        res.pop("results", None)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
