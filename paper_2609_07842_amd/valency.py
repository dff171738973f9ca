"""Valency control measured on the GPU: the mean number of neighbours within the attraction
range <z> and the fraction P_err of particles with more than f of them, against valency and
binding strength (Section 3, Fig. 2).

All conditions run side by side as replicas of one handle.  Binding strength beta E_a is
varied by scaling every energy of a replica by beta at kT = 1 (the Boltzmann weight
exp(-beta U) is the same as at temperature 1/beta; only the time unit changes), so one
integrator serves all conditions.  Strong binding condenses the dilute fluid into clusters,
so the layout holds local densities up to 1 (`rho_max`).

    python -m paper_2609_07842_amd.valency [--N 10000] [--steps 40000]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import vbc as _vbc
from . import workloads as W


def saturation_sweep(fs=(1, 2, 3, 4, 5, 6), beta_Ea=(1.0, 2.0, 4.0, 6.0, 8.0), N=10_000, rho=0.05,
                     E_a=2.0, steps=40_000, sample_every=2_000, precision="fp32", seed=31, log=None):
    say = log or (lambda m: None)
    conds = [(f, b) for f in fs for b in beta_Ea]
    L = W.box_length(N, rho)
    reps, xs, vs = [], [], []
    for k, (f, bE) in enumerate(conds):
        beta = bE / E_a
        p = W.vbc_params(E_r=20.0 * beta, E_a=E_a * beta, f=float(f))
        reps.append(_vbc.replica(N, L, p, seed=k))
        xs.append(W.uniform_positions(N, L, seed + k))
        vs.append(W.maxwell_boltzmann(N, 1.0, seed + 100 + k))
    s = _vbc.System(reps, precision=precision, rho_max=1.0)
    s.set_state(np.concatenate(xs), np.concatenate(vs))
    z_hist = {c: [] for c in conds}
    done = 0
    while done < steps:
        s.step(sample_every, integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=seed)
        done += sample_every
        s.check()
        if done > steps // 2:  # second half: sample
            _, _, sums = s.observables()
            sums = sums.cpu().numpy()
            for r, c in enumerate(conds):
                z_hist[c].append((sums[r, 0] / N, sums[r, 1] / N, sums[r, 2] / N))
        say(f"[valency] {done}/{steps} steps")
    out = {}
    for c in conds:
        h = np.array(z_hist[c])
        out[f"f={c[0]} betaEa={c[1]:g}"] = dict(f=c[0], beta_Ea=c[1], z=float(h[:, 0].mean()),
                                                 P_err=float(h[:, 1].mean()), penetrations=float(h[:, 2].mean()))
    return dict(workload=dict(N=N, rho=rho, E_a=E_a, steps=steps, precision=precision,
                              geometry="VBC(1.5, 2.0, 0)", integrator="Langevin gamma=0.1 dt=0.005"),
                results=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=10_000)
    ap.add_argument("--steps", type=int, default=40_000)
    a = ap.parse_args()
    res = saturation_sweep(N=a.N, steps=a.steps, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
