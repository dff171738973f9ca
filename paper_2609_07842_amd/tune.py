"""Autotuner of the layout knobs that change speed but no result beyond the rounding of
sums: the brick edge (cells per edge of the block of cells one workgroup owns, which sets
the LDS tile and the halo overhead) and the workgroup size of the brick kernels.

For a workload it times every candidate on the GPU (the start relaxed first, the step
graphs captured before the clock starts, then the median of three runs of whole steps
through the captured-graph path), discards candidates that do not fit the device's LDS
or overflow a capacity, and keeps the fastest in a JSON cache keyed by device name and
workload.  Each entry records the sha256 of the kernel source it was timed with;
`lookup` returns the cached choice only while that source is unchanged (else None, and
`stale` says why); `tune_fluid`, `tune_pool` and `tune_melt` fill the cache.

    python -m paper_2609_07842_amd.tune --N 1000000 --rho 0.5 --f 4 [--precision fp32]
    python -m paper_2609_07842_amd.tune --pool
    python -m paper_2609_07842_amd.tune --melt
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import time

from . import vbc as _vbc
from . import workloads as W

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
KERNEL_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "vbc_kernels.hip")


def kernel_hash():
    """sha256 of the kernel source the library is built from."""
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()
BRICKS = (2, 3, 4, 5)
BLOCKS = (128, 192, 256, 320, 384, 448, 512, 640, 768, 896, 1024)


def _device_name():
    """Architecture and compute-unit count of GPU 0, e.g. gfx950x256CU."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return f"{arch.split(':')[0]}x{p.multi_processor_count}CU"


def fluid_key(N, rho, precision, device=None):
    return f"{device or _device_name()}|fluid|N={int(N)}|rho={rho:g}|{precision}"


def pool_key(cfg, device=None):
    return (f"{device or _device_name()}|pool|rho={cfg.rho_max:g}|N={cfg.n_range[0]}-{cfg.n_range[1]}"
            f"|{cfg.precision}|tick={cfg.steps_per_tick}")


def melt_key(precision="fp32", device=None):
    return f"{device or _device_name()}|melt|N=1000000|rho=0.85|{precision}"


def load_cache(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_cache(cache, path=CACHE):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def stale(key, path=CACHE):
    """Why the cached entry for key is not used (None if it is)."""
    e = load_cache(path).get(key)
    if e is None:
        return "no entry"
    if e.get("kernel_sha256") != kernel_hash():
        return "timed with another kernel source"
    return None


def lookup(key, path=CACHE):
    """Cached {brick, block} for a key, or None if there is none or it was timed with
    another kernel source."""
    e = load_cache(path).get(key)
    if e is None or e.get("kernel_sha256") != kernel_hash():
        return None
    return dict(brick=e["brick"], block=e["block"])


def _time_fluid(wl, precision, brick, block, warmup, steps, skin, repeats=3):
    import torch
    s = _vbc.System(_vbc.replica(wl.N, wl.L, wl.params, skin=skin), precision=precision,
                    brick=brick, block=block)
    s.set_state(wl.x, wl.v)
    integ = dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=1)
    s.step(warmup, **integ)
    s.check()
    rates = []
    for _ in range(repeats):
        s.prepare_step(steps, **integ)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, **integ)
        torch.cuda.synchronize()
        rates.append(steps / (time.perf_counter() - t0))
    s.check()
    opts = s.options()
    s.close()
    return statistics.median(rates), opts


def tune_fluid(N=1_000_000, rho=0.5, f=4.0, precision="fp32", warmup=1500, steps=400,
               skin=W.SKIN, bricks=BRICKS, blocks=BLOCKS, path=CACHE, log=print):
    """Time every (brick, block) on one fluid replica; cache and return the fastest."""
    wl = W.fluid(N, rho, f, seed=11, precision=precision)
    results = []
    for brick in bricks:
        for block in blocks:
            try:
                sps, opts = _time_fluid(wl, precision, brick, block, warmup, steps, skin)
            except _vbc.VBCError as e:
                log(f"[tune] brick {brick} block {block}: skipped ({e})")
                continue
            results.append(dict(brick=brick, block=block, steps_per_s=sps, k_max=opts["k_max"],
                                stage_cap=opts["stage_cap"]))
            log(f"[tune] brick {brick} block {block}: {sps:.0f} steps/s")
    if not results:
        raise RuntimeError("no candidate layout fits")
    best = max(results, key=lambda r: r["steps_per_s"])
    cache = load_cache(path)
    cache[fluid_key(N, rho, precision)] = dict(best, workload=dict(N=N, rho=rho, f=f, skin=skin),
                                               candidates=results, kernel_sha256=kernel_hash())
    save_cache(cache, path)
    return best


def melt_system(wl, precision="fp32", **opts):
    """A handle for the bead-spring melt workload wl (chains of 50 beads, sticker types,
    harmonic bonds)."""
    return _vbc.System(_vbc.replica(wl.N, wl.L, wl.params, mask=wl.mask, chain_len=50,
                                    k_bond=wl.k_bond, r0_bond=wl.r0, skin=W.SKIN),
                       precision=precision, **opts)


def melt_integrator(wl):
    return dict(integrator="langevin", dt=wl.dt, kT=wl.kT, gamma=wl.gamma, seed=wl.seed)


def relaxed_melt(seed=4, warmup=1000, precision="fp32"):
    """The melt and its positions and velocities after `warmup` Langevin steps from the
    random-walk start, which packs beads at bond distance in overlapping chains: those steps
    run in a layout sized for local densities up to 2 with a long list (k_max 256)."""
    wl = W.polymer_melt(seed=seed, precision=precision)
    s = melt_system(wl, precision, brick=3, k_max=256, rho_max=2.0)
    s.set_state(wl.x, wl.v, types=wl.types)
    s.step(warmup, **melt_integrator(wl))
    s.check()
    x, v = (t.contiguous().clone() for t in s.get_state())
    s.close()
    return wl, x, v


def tune_melt(precision="fp32", steps=400, bricks=(3, 4), blocks=BLOCKS, path=CACHE, log=print):
    """Time every (brick, block) on the relaxed melt; cache and return the fastest."""
    import torch
    wl, x, v = relaxed_melt(precision=precision)
    integ = melt_integrator(wl)
    results = []
    for brick in bricks:
        for block in blocks:
            try:
                s = melt_system(wl, precision, brick=brick, block=block)
                s.set_state(x, v, types=wl.types)
                s.step(200, **integ)
                rates = []
                for _ in range(3):
                    s.prepare_step(steps, **integ)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s.step(steps, **integ)
                    torch.cuda.synchronize()
                    rates.append(steps / (time.perf_counter() - t0))
                s.check()
                opts = s.options()
                s.close()
            except _vbc.VBCError as e:
                log(f"[tune] melt brick {brick} block {block}: skipped ({e})")
                continue
            sps = statistics.median(rates)
            results.append(dict(brick=brick, block=block, steps_per_s=sps, k_max=opts["k_max"],
                                stage_cap=opts["stage_cap"]))
            log(f"[tune] melt brick {brick} block {block}: {sps:.0f} steps/s")
    if not results:
        raise RuntimeError("no candidate layout fits")
    best = max(results, key=lambda r: r["steps_per_s"])
    cache = load_cache(path)
    cache[melt_key(precision)] = dict(best, candidates=results, kernel_sha256=kernel_hash())
    save_cache(cache, path)
    return best


def tune_pool(cfg=None, n_requests=48, steps=200, blocks=BLOCKS, bricks=(3, 4, 5), path=CACHE,
              log=print):
    """Time a saturated request stream through the pool for every (brick, block)."""
    from . import serve
    cfg = cfg or serve.ServerConfig()
    reqs = serve.make_requests(n=n_requests, seed=17, rho=cfg.rho_max, steps=steps,
                               n_range=cfg.n_range)
    results = []
    for brick in bricks:
        for block in blocks:
            c = serve.ServerConfig(**{**cfg.__dict__, "brick": brick, "block": block})
            try:
                srv = serve.Server(c)
                r = srv.run(reqs)
                srv.pool.close()
            except _vbc.VBCError as e:
                log(f"[tune] pool brick {brick} block {block}: skipped ({e})")
                continue
            results.append(dict(brick=brick, block=block, particle_steps_per_s=r["particle_steps_per_s"],
                                step_p99_ms=r["step_latency_ms"]["p99"]))
            log(f"[tune] pool brick {brick} block {block}: {r['particle_steps_per_s']:.3g} particle-steps/s")
    if not results:
        raise RuntimeError("no candidate layout fits")
    best = max(results, key=lambda r: r["particle_steps_per_s"])
    cache = load_cache(path)
    cache[pool_key(cfg)] = dict(best, candidates=results, kernel_sha256=kernel_hash())
    save_cache(cache, path)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--rho", type=float, default=0.5)
    ap.add_argument("--f", type=float, default=4.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--pool", action="store_true", help="tune the serving pool instead")
    ap.add_argument("--melt", action="store_true", help="tune the bead-spring melt instead")
    ap.add_argument("--cache", default=CACHE, help="JSON cache to update")
    a = ap.parse_args()
    say = lambda m: print(m, flush=True)
    if a.pool:
        best = tune_pool(path=a.cache, log=say)
    elif a.melt:
        best = tune_melt(a.precision, path=a.cache, log=say)
    else:
        best = tune_fluid(a.N, a.rho, a.f, a.precision, path=a.cache, log=say)
    print(json.dumps(best), flush=True)


if __name__ == "__main__":
    main()
