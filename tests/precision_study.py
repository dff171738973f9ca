"""Precision study of the FP32-mixed path against FP64 and the oracle (test infrastructure).

Workload: N = 10^5 particles at density 0.3, standard VBC(1.5, 2.0, 0) geometry, well depth
5 kT, valency f = 1..6, Langevin kT = 1, gamma = 0.1, dt = 0.005, the same seeded start and
noise for both precisions.  Every `every` steps (and at t = 0) each run is evaluated once:

* forces of a random sample of particles against the FP64 oracle at the run's own positions
  (normwise relative error max_i |dF_i| / max_i |F_i| over the sample);
* the trajectory observables U/N (from the library's FP64 energy reduction), the mean
  number z of neighbours within r_a and the fraction P_err of particles with more than f
  of them (Section 3's measures of valency control), counted on the host from the state.

FP32 and FP64 trajectories separate (the dynamics are chaotic), so they are compared
through these statistics, not point by point.  Strong valency-limited attraction makes the
fluid condense locally, so the layout is sized to hold local densities up to 1.0
(`rho_max`) rather than margins around the mean density.

    python tests/precision_study.py [--N 100000] [--steps 10000] [--every 2000] [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2609_07842_amd import workloads as W  # noqa: E402


def neighbour_stats(x, L, r_a, f):
    from scipy.spatial import cKDTree
    tree = cKDTree(np.mod(x, L), boxsize=L)
    z = np.array([len(v) - 1 for v in tree.query_ball_point(np.mod(x, L), r_a)])
    return float(z.mean()), float((z > f).mean())


def run_one(N, rho, f, steps, every, sample, seed, precision, log=print):
    import torch
    from paper_2609_07842_amd import vbc
    wl = W.fluid(N, rho, f, E_a=5.0, seed=seed, precision=precision)
    p = wl.params
    s = vbc.System(vbc.replica(wl.N, wl.L, p), precision=precision, rho_max=1.0)
    s.set_state(wl.x, wl.v)
    rng = np.random.default_rng(seed + 7)
    snaps = []
    t_steps = 0.0
    done = 0
    while True:
        F, e, UW = s.force()
        s.check()
        x = s.get_state()[0].cpu().numpy()
        Fg = F.cpu().numpy()
        idx = np.sort(rng.choice(N, size=sample, replace=False))
        ref = oracle.evaluate_subset(x, wl.L, p, idx)["F"]
        err = float(np.linalg.norm(Fg[idx] - ref, axis=1).max() / np.linalg.norm(ref, axis=1).max())
        z, perr = neighbour_stats(x, wl.L, p["r_a"], f)
        U = float(UW.cpu().numpy()[0, 0])
        snaps.append(dict(step=done, force_err=err, U_per_N=U / N, z=z, P_err=perr))
        log(f"  f={f:g} {precision} step {done}: |dF|/|F| {err:.2e}  U/N {U / N:.4f}  z {z:.3f}  P_err {perr:.4f}")
        if done >= steps:
            break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(every, integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=seed)
        torch.cuda.synchronize()
        t_steps += time.perf_counter() - t0
        done += every
    s.check()
    return dict(snapshots=snaps, steps_per_s=(steps / t_steps) if t_steps else None)


def study(N=100_000, rho=0.3, fs=(1, 2, 3, 4, 5, 6), steps=10_000, every=2_000, sample=256, seed=21,
          log=print):
    out = dict(workload=dict(N=N, rho=rho, E_a=5.0, geometry="VBC(1.5, 2.0, 0)", integrator="Langevin kT=1 gamma=0.1 dt=0.005",
                             steps=steps, every=every, sample=sample, seed=seed), results={})
    for f in fs:
        r = {prec: run_one(N, rho, f, steps, every, sample, seed, prec, log) for prec in ("fp64", "fp32")}
        a, b = r["fp64"]["snapshots"], r["fp32"]["snapshots"]
        late = slice(1, None) if len(a) > 1 else slice(0, None)
        mean = lambda s, k: float(np.mean([q[k] for q in s[late]]))
        r["compare"] = dict(
            max_force_err_fp64=max(q["force_err"] for q in a),
            max_force_err_fp32=max(q["force_err"] for q in b),
            U_per_N=(mean(a, "U_per_N"), mean(b, "U_per_N")),
            z=(mean(a, "z"), mean(b, "z")),
            P_err=(mean(a, "P_err"), mean(b, "P_err")))
        out["results"][str(f)] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=100_000)
    ap.add_argument("--steps", type=int, default=10_000)
    ap.add_argument("--every", type=int, default=2_000)
    ap.add_argument("--sample", type=int, default=256)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = study(N=a.N, steps=a.steps, every=a.every, sample=a.sample,
                log=lambda m: print(m, flush=True))
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    print(json.dumps({f: v["compare"] for f, v in res["results"].items()}), flush=True)


if __name__ == "__main__":
    main()
