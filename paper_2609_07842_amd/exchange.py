"""Energy landscape of the partner exchange (Section 4): a centre saturated with f bonds
trades one partner for a free particle, all three on one line.  The centre sits at the
origin with f - 1 spectator partners at the well minimum m = (r_r + r_a) / 2 on +y, -y, +z,
-z (so f <= 5); the leaving partner A sits at +r_A and the newcomer B at -r_B on the x axis.
U(r_A, r_B) is evaluated on a square grid of both distances from 0.9 r_r to
d = max(r_a, r_h) + 0.5, beyond every range of the potential.

* The two bonded states are the minima of U(r_A, d) (A bonded, B away) and of U(d, r_B);
  they are equal by symmetry.
* The exchange barrier is the height, above that minimum, of the lowest path between them
  on the grid: the minimax (bottleneck) path, found by adding grid points in order of
  energy until the two states connect.
* A trap is a grid state with both A and B well inside the attractive well (closer than
  m + w / 2, w = (r_a - r_r) / 2: at least about half the well depth each) that lies below
  the bonded state by more than 1 % of E_a: an extra particle bound to an already saturated
  centre.  (At the edge of the range, r -> r_a, the newcomer barely interacts and such
  states are degenerate with the bonded one; they are not traps.)

Every grid point is one replica of a batched handle, so a whole landscape is one force
evaluation per 1024 points on the GPU.

    python -m paper_2609_07842_amd.exchange [--points 41]
"""
from __future__ import annotations

import argparse
import itertools
import json

import numpy as np

from . import vbc as _vbc
from . import workloads as W

SPECTATORS = np.array([[0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
BOX = 24.0


def grid_radii(params, points):
    d = max(params["r_a"], params["r_h"]) + 0.5
    return np.linspace(0.9 * params["r_r"], d, points)


def positions(params, f, r_A, r_B):
    """Positions (f + 2, 3), shifted to the box centre: centre, A, B, then the f - 1
    spectators."""
    if not 1 <= f <= 5:
        raise ValueError("the spectators cover at most four directions: f must be 1..5")
    m = 0.5 * (params["r_r"] + params["r_a"])
    x = np.zeros((f + 2, 3))
    x[1, 0] = r_A
    x[2, 0] = -r_B
    x[3:] = m * SPECTATORS[:f - 1]
    return x + BOX / 2


def landscapes(geoms, fs, points=41, E_a=2.0, precision="fp64"):
    """U(r_A, r_B) for every (geometry, f), geoms a list of (r_l, r_h, delta): array
    [len(geoms), len(fs), points, points] and the radii of each geometry."""
    radii, jobs = [], []
    for g in geoms:
        p = W.vbc_params(E_a=E_a, r_l=g[0], r_h=g[1], delta=g[2])
        r = grid_radii(p, points)
        radii.append(r)
        for f in fs:
            for a in r:
                for b in r:
                    jobs.append((g, f, a, b))
    U = np.empty(len(jobs))
    for c0 in range(0, len(jobs), 1024):
        chunk = jobs[c0:c0 + 1024]
        reps, xs = [], []
        for (rl, rh, dl), f, a, b in chunk:
            p = W.vbc_params(E_a=E_a, f=float(f), r_l=rl, r_h=rh, delta=dl)
            reps.append(_vbc.replica(f + 2, BOX, p))
            xs.append(positions(p, f, a, b))
        s = _vbc.System(reps, precision=precision)
        s.set_state(np.concatenate(xs))
        _, _, UW = s.force()
        s.check()
        U[c0:c0 + len(chunk)] = UW.cpu().numpy()[:len(chunk), 0]
        s.close()
    return U.reshape(len(geoms), len(fs), points, points), radii


def bottleneck(U, src, dst):
    """Lowest possible maximum of U along a path between grid points src and dst (steps to
    the 8 neighbours): points are added in order of energy, joined by union-find, until src
    and dst are connected."""
    n0, n1 = U.shape
    parent = np.arange(n0 * n1)

    def find(k):
        while parent[k] != k:
            parent[k] = parent[parent[k]]
            k = parent[k]
        return k

    on = np.zeros(n0 * n1, dtype=bool)
    s, t = src[0] * n1 + src[1], dst[0] * n1 + dst[1]
    for k in np.argsort(U, axis=None, kind="stable"):
        on[k] = True
        i, j = divmod(int(k), n1)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                a, b = i + di, j + dj
                if (di or dj) and 0 <= a < n0 and 0 <= b < n1 and on[a * n1 + b]:
                    ra, rb = find(k), find(a * n1 + b)
                    if ra != rb:
                        parent[ra] = rb
        if on[s] and on[t] and find(s) == find(t):
            return float(U.flat[k])
    return float("inf")


def barrier_and_trap(U, r, r_r=1.0, r_a=1.5, E_a=2.0):
    """(barrier above the bonded state, trap present) of one landscape U[r_A, r_B]."""
    far = len(r) - 1
    ia = int(np.argmin(U[:, far]))          # A bonded, B away
    ib = int(np.argmin(U[far, :]))          # B bonded, A away
    u0 = min(U[ia, far], U[far, ib])
    saddle = bottleneck(U, (ia, far), (far, ib))
    w = 0.5 * (r_a - r_r)
    core = r < 0.5 * (r_r + r_a) + 0.5 * w
    both = core[:, None] & core[None, :]
    trap = bool(np.any(U[both] < u0 - 0.01 * E_a))
    return saddle - u0, trap


def scan(r_l=(1.20, 1.25, 1.29, 1.35, 1.40, 1.45), r_h=(1.50, 1.60, 1.70, 1.80, 1.90, 2.00),
         delta=(0.0, 0.15, 0.30, 0.45), fs=(1, 2, 3, 4, 5), points=21, E_a=2.0, r_a=1.5):
    """Barrier of every geometry r_l < r_h of the grid at every valency; the objective is the
    worst barrier over the valencies among geometries without a trap at any of them.  The
    counting range must cover the attraction range (r_h >= r_a): a particle attracted
    beyond r_h would bind without being counted."""
    geoms = [g for g in itertools.product(r_l, r_h, delta) if g[0] < g[1] and g[1] >= r_a]
    U, radii = landscapes(geoms, fs, points, E_a)
    rows = []
    for k, g in enumerate(geoms):
        bt = [barrier_and_trap(U[k, j], radii[k], E_a=E_a) for j in range(len(fs))]
        rows.append(dict(r_l=g[0], r_h=g[1], delta=g[2], barriers=[b for b, _ in bt],
                         trap=any(t for _, t in bt), worst=max(b for b, _ in bt)))
    ok = [r for r in rows if not r["trap"]]
    ok.sort(key=lambda r: r["worst"])
    return dict(E_a=E_a, valencies=list(fs), points=points, geometries=len(rows), trap_free=len(ok),
                best=ok[:5], rows=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--points", type=int, default=41)
    a = ap.parse_args()
    named = {"standard VBC(1.5, 2.0, 0)": (1.5, 2.0, 0.0),
             "exchange-tuned VBC(1.29, 1.50, 0.30)": (1.29, 1.50, 0.30)}
    U, radii = landscapes(list(named.values()), (1, 2, 3, 4, 5), a.points)
    out = {"named": {name: [barrier_and_trap(U[k, j], radii[k]) for j in range(5)]
                     for k, name in enumerate(named)}}
    res = scan()
    res.pop("rows")
    out["scan"] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
