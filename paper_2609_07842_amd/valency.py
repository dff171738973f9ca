"""Valency control measured on the GPU: the mean number of neighbours within the attraction
range <z> and the fraction P_err of particles with more than f of them, against valency and
binding strength (Section 3, Fig. 2), with the connectivity of the bond graph: the giant
component P_inf, the fraction x_cyc of particles in loop-carrying clusters, and the
cluster-size distributions of all and of acyclic clusters next to the Flory-Stockmayer
density of tree clusters, eq. (fs), at the measured saturation p = <z>/f (Figs. 3-5).

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
import math
import sys

import numpy as np

from . import vbc as _vbc
from . import workloads as W


def fs_density(s, f, p, rho):
    """Flory-Stockmayer number density of tree clusters of size s, eq. (fs):
    rho w_s (1 - p)^f [p (1 - p)^(f - 2)]^(s - 1) with w_s = f (fs - s)! / ((fs - 2s + 2)! s!),
    evaluated through log-factorials."""
    if p <= 0.0:
        return rho if s == 1 else 0.0
    if p >= 1.0:
        return 0.0
    if (f - 2) * s + 2 < 0:
        return 0.0  # 1 / (negative integer)! = 0: a tree of s needs s - 1 <= f s / 2 bonds
    log_w = math.log(f) + math.lgamma((f - 1) * s + 1) - math.lgamma((f - 2) * s + 3) - math.lgamma(s + 1)
    log_t = f * math.log1p(-p) + (s - 1) * (math.log(p) + (f - 2) * math.log1p(-p))
    return rho * math.exp(log_w + log_t)


def saturation_sweep(fs=(1, 2, 3, 4, 5, 6), beta_Ea=(1.0, 2.0, 4.0, 6.0, 8.0), N=10_000, rho=0.05,
                     E_a=2.0, steps=40_000, sample_every=2_000, precision="fp32", seed=31, log=None,
                     hist_len=64):
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
    c_hist = {c: [] for c in conds}
    sizes = np.zeros((len(conds), 2, hist_len), dtype=np.int64)
    nsamp = 0
    done = 0
    while done < steps:
        s.step(sample_every, integrator="langevin", dt=0.005, kT=1.0, gamma=0.1, seed=seed)
        done += sample_every
        s.check()
        if done > steps // 2:  # second half: sample
            _, _, sums = s.observables()
            _, cst, hist = s.clusters(hist_len=hist_len, labels=False)
            sums, cst = sums.cpu().numpy(), cst.cpu().numpy()
            sizes += hist.cpu().numpy()[:len(conds)]
            nsamp += 1
            for r, c in enumerate(conds):
                z_hist[c].append((sums[r, 0] / N, sums[r, 1] / N, sums[r, 2] / N))
                c_hist[c].append((cst[r, 1] / N, cst[r, 2] / N, cst[r, 0] / N))
        say(f"[valency] {done}/{steps} steps")
    out = {}
    V = float(L) ** 3
    for k, c in enumerate(conds):
        h = np.array(z_hist[c])
        g = np.array(c_hist[c])
        z = float(h[:, 0].mean())
        p_sat = z / c[0]
        # number densities of clusters of size s (index 0: sizes >= hist_len), sample mean
        dens_all = sizes[k, 0] / (nsamp * V)
        dens_acyc = sizes[k, 1] / (nsamp * V)
        fs_pred = [fs_density(m, c[0], p_sat, rho) if m > 0 else None for m in range(hist_len)]
        out[f"f={c[0]} betaEa={c[1]:g}"] = dict(
            f=c[0], beta_Ea=c[1], z=z, P_err=float(h[:, 1].mean()), penetrations=float(h[:, 2].mean()),
            saturation=p_sat, P_inf=float(g[:, 0].mean()), x_cyc=float(g[:, 1].mean()),
            clusters_per_particle=float(g[:, 2].mean()),
            rho_s_all=dens_all.tolist(), rho_s_acyclic=dens_acyc.tolist(), rho_s_fs=fs_pred)
    return dict(workload=dict(N=N, rho=rho, E_a=E_a, steps=steps, precision=precision,
                              geometry="VBC(1.5, 2.0, 0)", integrator="Langevin gamma=0.1 dt=0.005"),
                results=out)


STABILITY_EA = (0.1, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0)


def stability_sweep(E_as=STABILITY_EA, geometries=("standard", "partial", "blind", "none"), N=1000,
                    rho=0.05, steps=200_000, sample_every=1_000, dt=0.01, precision="fp32", seed=41,
                    rho_max=3.0, log=None):
    """The stability study of Section 6.2 (Fig. 12): the four counter geometries of
    workloads.stability_sets (standard VBC(1.5, 2.0) with f = 12, partial coverage
    r_h = 1.25 with f = 0.5, blind coverage r_h = 1.0 with f = 0.001, and no correction,
    f = 1000) at N = 1000, density 0.05, E_r = 20, r_r = 1, r_a = 1.5, over a sweep of the
    well depth E_a; Langevin kT = 1, gamma = 0.1, dt = 0.01.  Every (geometry, E_a) pair is
    a replica of one handle laid out for the collapsed droplets of the uncorrected system
    (local densities up to rho_max, bricks of 2^3 cells to keep that staging in LDS).  Over
    the second half of the run, sampled every `sample_every` steps: the mean number of
    neighbours within r_a per particle (contacts, panel (a)) and within r_r (core
    penetrations, panel (b)), with the interquartile range across frames."""
    say = log or (lambda m: None)
    conds = [(g, e) for g in geometries for e in E_as]
    L = W.box_length(N, rho)
    reps, xs, vs = [], [], []
    for k, (g, e) in enumerate(conds):
        reps.append(_vbc.replica(N, L, W.stability_sets(e)[g], seed=k))
        xs.append(W.uniform_positions(N, L, seed + k))
        vs.append(W.maxwell_boltzmann(N, 1.0, seed + 100 + k))
    s = _vbc.System(reps, precision=precision, rho_max=rho_max, brick=2)
    s.set_state(np.concatenate(xs), np.concatenate(vs))
    frames = {c: [] for c in conds}
    done = 0
    while done < steps:
        s.step(sample_every, integrator="langevin", dt=dt, kT=1.0, gamma=0.1, seed=seed)
        done += sample_every
        if done > steps // 2:
            _, _, sums = s.observables()
            sums = sums.cpu().numpy()
            for r, c in enumerate(conds):
                frames[c].append((sums[r, 0] / N, sums[r, 2] / N))
        if done % (10 * sample_every) == 0:
            s.check()
            say(f"[stability] {done}/{steps} steps")
    s.check()
    s.close()
    out = {}
    for c in conds:
        h = np.array(frames[c])
        out.setdefault(c[0], {})[f"{c[1]:g}"] = dict(
            contacts=float(h[:, 0].mean()), contacts_iqr=[float(np.percentile(h[:, 0], 25)),
                                                         float(np.percentile(h[:, 0], 75))],
            penetrations=float(h[:, 1].mean()), penetrations_iqr=[float(np.percentile(h[:, 1], 25)),
                                                                 float(np.percentile(h[:, 1], 75))])
    return dict(workload=dict(N=N, rho=rho, E_r=20.0, r_r=1.0, r_a=1.5, steps=steps, dt=dt,
                              precision=precision, integrator="Langevin kT=1 gamma=0.1",
                              sampled="second half, every %d steps" % sample_every),
                results=out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=10_000)
    ap.add_argument("--steps", type=int, default=40_000)
    ap.add_argument("--stability", action="store_true",
                    help="run the stability sweep of the four counter geometries instead")
    a = ap.parse_args()
    say = lambda m: print(m, file=sys.stderr, flush=True)
    if a.stability:
        res = stability_sweep(log=say)
    else:
        res = saturation_sweep(N=a.N, steps=a.steps, log=say)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
