"""Energy along the partner-exchange path (Section 4): a centre saturated with f bonds
trades one partner for a free particle, all three on one line.  The centre sits at the
origin with f - 1 spectator partners at the well minimum m = (r_r + r_a) / 2 on +y, -y, +z,
-z (so f <= 5); partner A starts at +m on the x axis and the newcomer B at -d, beyond every
range of the potential (d = max(r_a, r_h) + 0.5).  Along the path (lambda from 0 to 1) A moves
out to +d and B in to -m, both linearly, so the path is symmetric (U(0) = U(1)).

The barrier is max U(lambda) - U(0).  A trap is a local minimum of U strictly inside the
path that lies below U(0): a bound state of the saturated centre with an extra particle.
Every point of the path is one replica of a single handle, so a scan over geometries is a
few force evaluations on the GPU.

    python -m paper_2609_07842_amd.exchange [--points 81]
"""
from __future__ import annotations

import argparse
import itertools
import json
import sys

import numpy as np

from . import vbc as _vbc
from . import workloads as W

SPECTATORS = np.array([[0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
BOX = 24.0


def path_positions(params, f, lam):
    """Positions (f + 2, 3) at path parameter lam, shifted to the box centre: centre, A, B,
    then the f - 1 spectators."""
    if not 1 <= f <= 5:
        raise ValueError("the path places at most four spectators: f must be 1..5")
    m = 0.5 * (params["r_r"] + params["r_a"])
    d = max(params["r_a"], params["r_h"]) + 0.5
    x = np.zeros((f + 2, 3))
    x[1, 0] = m + lam * (d - m)
    x[2, 0] = -(d - lam * (d - m))
    x[3:] = m * SPECTATORS[:f - 1]
    return x + BOX / 2


def profiles(geoms, fs, points=81, E_a=2.0, precision="fp64"):
    """U(lambda) for every (geometry, f): geoms is a list of (r_l, r_h, delta).  Returns an
    array [len(geoms), len(fs), points]."""
    lams = np.linspace(0.0, 1.0, points)
    jobs = [(g, f, lam) for g in geoms for f in fs for lam in lams]
    U = np.empty(len(jobs))
    for c0 in range(0, len(jobs), 1024):
        chunk = jobs[c0:c0 + 1024]
        reps, xs = [], []
        for (rl, rh, dl), f, lam in chunk:
            p = W.vbc_params(E_a=E_a, f=float(f), r_l=rl, r_h=rh, delta=dl)
            reps.append(_vbc.replica(f + 2, BOX, p))
            xs.append(path_positions(p, f, lam))
        s = _vbc.System(reps, precision=precision)
        s.set_state(np.concatenate(xs))
        _, _, UW = s.force()
        s.check()
        U[c0:c0 + len(chunk)] = UW.cpu().numpy()[:len(chunk), 0]
        s.close()
    return U.reshape(len(geoms), len(fs), points)


def barrier_and_trap(u):
    """Barrier max U - U(0) and whether a local minimum inside the path lies below U(0)."""
    inner = u[1:-1]
    is_min = (inner < u[:-2]) & (inner <= u[2:])
    trap = bool(np.any(is_min & (inner < u[0] - 1e-12)))
    return float(u.max() - u[0]), trap


def scan(r_l=np.round(np.arange(1.20, 1.51, 0.03), 2), r_h=np.round(np.arange(1.40, 2.01, 0.05), 2),
         delta=(0.0, 0.1, 0.2, 0.3, 0.4), fs=(1, 2, 3, 4, 5), points=41, E_a=2.0):
    """Barrier of every geometry r_l < r_h in the grid at every valency; the objective is the
    worst barrier over the valencies, geometries with a trap at any valency excluded."""
    geoms = [g for g in itertools.product(r_l, r_h, delta) if g[0] < g[1]]
    U = profiles(geoms, fs, points, E_a)
    rows = []
    for k, g in enumerate(geoms):
        bt = [barrier_and_trap(U[k, j]) for j in range(len(fs))]
        rows.append(dict(r_l=float(g[0]), r_h=float(g[1]), delta=float(g[2]),
                         barriers=[b for b, _ in bt], trap=any(t for _, t in bt),
                         worst=max(b for b, _ in bt)))
    ok = [r for r in rows if not r["trap"]]
    best = min(ok, key=lambda r: r["worst"]) if ok else None
    return dict(E_a=E_a, valencies=list(fs), points=points, geometries=len(rows), best=best, rows=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=41)
    a = ap.parse_args()
    res = scan(points=a.points)
    named = {"standard VBC(1.5, 2.0, 0)": (1.5, 2.0, 0.0), "exchange-tuned VBC(1.29, 1.50, 0.30)": (1.29, 1.50, 0.30)}
    U = profiles(list(named.values()), (1, 2, 3, 4, 5), a.points)
    res["named"] = {name: [barrier_and_trap(U[k, j]) for j in range(5)] for k, name in enumerate(named)}
    res.pop("rows")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
