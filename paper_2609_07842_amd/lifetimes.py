"""Bond lifetimes against saturation on the GPU (Section 4, Fig. 7): the median lifetime
of a bond (r_ij < r_a, followed from the sample at which it first appears to the first
sample without it) for the standard VBC(1.5, 2.0, 0) and the exchange-tuned
VBC(1.29, 1.50, 0.30), at valencies 1 and 2 where both run with dt = 0.01 (the step rule of
Section 4), over a range of binding strengths.

All conditions run side by side as replicas of one handle; binding strength beta E_a is set
by scaling every energy of a replica by beta at kT = 1 (same Boltzmann weight as
temperature 1/beta).  After `equil` steps the tracker is reset, then sampled every `every`
steps for `steps` steps; lifetimes are in steps (units of dt), with the sampling interval
as resolution, and the saturation is p = <z>/f averaged over the samples.  Two estimates:
tau_median, the median of the bonds that formed and broke inside the window (biased to
short lifetimes when many bonds outlive the window), and tau_rate, the bond time summed
over the window divided by the number of bonds that broke in it (the maximum-likelihood
mean of exponential lifetimes under censoring).

    python -m paper_2609_07842_amd.lifetimes [--N 4000] [--steps 40000]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import vbc as _vbc
from . import workloads as W

GEOMETRIES = {"standard": dict(r_l=1.5, r_h=2.0, delta=0.0), "exchange": dict(r_l=1.29, r_h=1.50, delta=0.30)}


def lifetime_sweep(geometries=("standard", "exchange"), fs=(1, 2), beta_Ea=(1.0, 2.0, 4.0, 6.0, 8.0),
                   N=4000, rho=0.05, E_a=2.0, equil=20_000, steps=40_000, every=10, precision="fp32",
                   seed=41, log=None):
    say = log or (lambda m: None)
    dts = {W.exchange_dt(f) for f in fs}
    if len(dts) != 1:
        raise ValueError("valencies with different time steps cannot share one integrator call")
    dt = dts.pop()
    conds = [(g, f, b) for g in geometries for f in fs for b in beta_Ea]
    L = W.box_length(N, rho)
    reps, xs, vs = [], [], []
    for k, (g, f, bE) in enumerate(conds):
        beta = bE / E_a
        p = W.vbc_params(E_r=20.0 * beta, E_a=E_a * beta, f=float(f), **GEOMETRIES[g])
        reps.append(_vbc.replica(N, L, p, seed=k))
        xs.append(W.uniform_positions(N, L, seed + k))
        vs.append(W.maxwell_boltzmann(N, 1.0, seed + 100 + k))
    s = _vbc.System(reps, precision=precision, rho_max=1.0)
    s.set_state(np.concatenate(xs), np.concatenate(vs))
    integ = dict(integrator="langevin", dt=dt, kT=1.0, gamma=0.1, seed=seed)
    done = 0
    while done < equil:
        k = min(2000, equil - done)
        s.step(k, **integ)
        done += k
    s.check()
    say(f"[lifetimes] equilibrated {equil} steps")
    tr = s.bond_tracker(max_partners=16, hist_len=steps // every + 2, bin_steps=every)
    zsum = np.zeros(len(conds))
    nz = 0
    done = 0
    while done < steps:
        s.step(every, **integ)
        done += every
        tr.sample()
        if done % (50 * every) == 0:
            _, _, sums = s.observables()
            zsum += sums.cpu().numpy()[:len(conds), 0] / N
            nz += 1
        if done % 10_000 == 0:
            say(f"[lifetimes] {done}/{steps} steps")
    s.check()
    stats = tr.stats.cpu().numpy()
    out = {}
    for r, (g, f, bE) in enumerate(conds):
        z = float(zsum[r] / max(nz, 1))
        out[f"{g} f={f} betaEa={bE:g}"] = dict(
            geometry=g, f=f, beta_Ea=bE, saturation=z / f, tau_median=tr.median_lifetime(r),
            tau_rate=(float(stats[r, 4] * every / (stats[r, 1] + stats[r, 2]))
                      if stats[r, 1] + stats[r, 2] else None),
            formed=int(stats[r, 0]), broken=int(stats[r, 1]), censored=int(stats[r, 2]),
            overflow=int(stats[r, 3]))
    return dict(workload=dict(N=N, rho=rho, E_a=E_a, dt=dt, equil=equil, steps=steps, every=every,
                              precision=precision, integrator="Langevin gamma=0.1"), results=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=4000)
    ap.add_argument("--equil", type=int, default=20_000)
    ap.add_argument("--steps", type=int, default=40_000)
    a = ap.parse_args()
    res = lifetime_sweep(N=a.N, equil=a.equil, steps=a.steps,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
