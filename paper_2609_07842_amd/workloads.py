"""Seeded synthetic inputs for the VBC hot path.

This module holds only input generation: positions, velocities, types, chain
topology, parameter presets and request streams.  It contains none of the
method's arithmetic, so both the GPU path and the FP64 oracle can be fed from it.

All workloads are synthetic (the paper uses no public dataset): uniform random
positions in a cubic periodic box at the stated number density, Maxwell-Boltzmann
velocities at kT, and bead-spring chains built as random walks of unit steps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Parameter presets (Section 2: polynomial soft-core potential, standard VBC)
# ---------------------------------------------------------------------------


def vbc_params(E_r=20.0, r_r=1.0, E_a=2.0, r_a=1.5, r_l=1.5, r_h=2.0, f=1.0, delta=0.0):
    """One type-pair entry.  Defaults: the standard VBC(1.5, 2.0, 0) with the paper's
    default soft-core parameters (Section 2, end of the general formulation)."""
    return dict(E_r=float(E_r), r_r=float(r_r), E_a=float(E_a), r_a=float(r_a),
                r_l=float(r_l), r_h=float(r_h), f=float(f), delta=float(delta))


def exchange_tuned(**kw):
    """VBC(1.29, 1.50, 0.30): the exchange-optimised geometry of Section 4."""
    base = dict(r_l=1.29, r_h=1.50, delta=0.30)
    base.update(kw)
    return vbc_params(**base)


def exchange_dt(f):
    """Time step for the exchange-tuned geometry (Section 4): 0.01 for valencies 1 and 2 (as
    for the standard geometry), 0.005 from valency 3 on, where the steeper switching of
    VBC(1.29, 1.50, 0.30) needs the shorter step."""
    return 0.01 if f <= 2 else 0.005


def stability_sets(E_a=1.0):
    """The four counter geometries compared in the stability study (Section 6.2)."""
    return {
        "standard": vbc_params(E_a=E_a, r_l=1.5, r_h=2.0, f=12.0),
        "partial": vbc_params(E_a=E_a, r_l=0.75, r_h=1.25, f=0.5),
        "blind": vbc_params(E_a=E_a, r_l=0.5, r_h=1.0, f=0.001),
        "none": vbc_params(E_a=E_a, r_l=1.5, r_h=2.0, f=1000.0),
    }


SKIN = 0.4  # neighbour-list buffer used by the paper's benchmarks (Section 5)

# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------


def box_length(N: int, rho: float) -> float:
    return (N / rho) ** (1.0 / 3.0)


def uniform_positions(N: int, L, seed: int) -> np.ndarray:
    """N x 3 positions uniform in [0, L)^3 (float64)."""
    rng = np.random.default_rng(seed)
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    x = rng.random((N, 3)) * Lv
    # guard the half-open interval against rounding up to L
    x = np.where(x >= Lv, 0.0, x)
    return x


def maxwell_boltzmann(N: int, kT: float, seed: int, remove_com: bool = True) -> np.ndarray:
    """N x 3 velocities, unit masses, normal with variance kT; centre-of-mass removed."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, math.sqrt(kT), size=(N, 3))
    if remove_com and N > 0:
        v -= v.mean(axis=0, keepdims=True)
    return v


def random_walk_chains(nchains: int, nbeads: int, L: float, seed: int, bond: float = 1.0):
    """Bead-spring chains as random walks of fixed step `bond` from uniform random
    starts, wrapped into [0, L)^3.  Returns positions (N x 3), bonds (B x 2, consecutive
    beads of one chain) and the bead index within its chain."""
    rng = np.random.default_rng(seed)
    starts = rng.random((nchains, 1, 3)) * L
    steps = rng.normal(size=(nchains, nbeads - 1, 3))
    steps /= np.linalg.norm(steps, axis=2, keepdims=True)
    steps *= bond
    walk = np.concatenate([np.zeros((nchains, 1, 3)), np.cumsum(steps, axis=1)], axis=1)
    x = (starts + walk).reshape(-1, 3)
    x = np.mod(x, L)
    x = np.where(x >= L, 0.0, x)
    bead = np.tile(np.arange(nbeads), nchains)
    base = (np.arange(nchains) * nbeads)[:, None] + np.arange(nbeads - 1)[None, :]
    bonds = np.stack([base.ravel(), base.ravel() + 1], axis=1).astype(np.int64)
    return x, bonds, bead


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    N: int
    L: float
    x: np.ndarray
    v: np.ndarray
    params: object  # dict (one type) or list of ntypes^2 dicts
    types: np.ndarray | None = None
    mask: np.ndarray | None = None
    bonds: np.ndarray | None = None
    k_bond: float = 0.0
    r0: float = 1.0
    precision: str = "fp64"
    integrator: str = "nve"
    dt: float = 0.005
    kT: float = 1.0
    gamma: float = 0.1
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def ntypes(self) -> int:
        return 1 if isinstance(self.params, dict) else int(round(len(self.params) ** 0.5))


def small_fluid(N=1000, rho=0.3, f=2.0, E_a=5.0, seed=1, precision="fp64", integrator="nve"):
    """N = 1000 at density 0.3, standard geometry, well depth 5 kT, valency 2, FP64,
    velocity-Verlet at dt = 0.005 (the small single-GPU case)."""
    L = box_length(N, rho)
    return Workload(
        name=f"fluid_N{N}_rho{rho}_f{f:g}", N=N, L=L, x=uniform_positions(N, L, seed),
        v=maxwell_boltzmann(N, 1.0, seed + 1000), params=vbc_params(E_a=E_a, f=f),
        precision=precision, integrator=integrator, seed=seed,
        meta=dict(rho=rho, f=f, E_a=E_a))


def fluid(N, rho, f, E_a=5.0, seed=2, precision="fp32", integrator="langevin", **pkw):
    L = box_length(N, rho)
    return Workload(
        name=f"fluid_N{N}_rho{rho}_f{f:g}", N=N, L=L, x=uniform_positions(N, L, seed),
        v=maxwell_boltzmann(N, 1.0, seed + 1000), params=vbc_params(E_a=E_a, f=f, **pkw),
        precision=precision, integrator=integrator, seed=seed,
        meta=dict(rho=rho, f=f, E_a=E_a))


def headline(f=4.0, seed=3):
    """N = 10^6 at density 0.5, valency 4, well depth 5 kT, standard geometry, FP32
    pair arithmetic with FP64 integration, Langevin kT = 1, dt = 0.005."""
    return fluid(1_000_000, 0.5, f, E_a=5.0, seed=seed)


def polymer_melt(nchains=20000, nbeads=50, rho=0.85, E_a=8.0, sticker_every=5, seed=4,
                 precision="fp32"):
    """Bead-spring melt: harmonic bonds k = 100, r0 = 1; every fifth bead (index 4 mod 5)
    is a valency-1 sticker with well depth E_a that counts only stickers; all other
    pairs are soft-core repulsion only."""
    N = nchains * nbeads
    L = box_length(N, rho)
    x, bonds, bead = random_walk_chains(nchains, nbeads, L, seed)
    types = (bead % sticker_every == sticker_every - 1).astype(np.int32)
    inert = vbc_params(E_a=0.0, f=1.0)
    sticky = vbc_params(E_a=E_a, f=1.0)
    params = [inert, inert, inert, sticky]  # (0,0) (0,1) (1,0) (1,1)
    mask = np.array([0b00, 0b10], dtype=np.uint32)  # type 0 counts nothing, stickers count stickers
    return Workload(
        name=f"melt_{nchains}x{nbeads}_rho{rho}", N=N, L=L, x=x,
        v=maxwell_boltzmann(N, 1.0, seed + 1000), params=params, types=types, mask=mask,
        bonds=bonds, k_bond=100.0, r0=1.0, precision=precision, integrator="langevin",
        seed=seed, meta=dict(rho=rho, nchains=nchains, nbeads=nbeads, E_a=E_a))


def serving_requests(n=256, seed=5, rho=0.3, N_min=1_000, N_max=200_000, steps=1000):
    """Request stream: N log-uniform in [N_min, N_max], valency uniform in 1..6, well
    depth uniform in [2, 10] kT, 1000 steps each.  Arrival times are drawn by the
    caller from the rate it targets; here only unit-rate exponential gaps are drawn."""
    rng = np.random.default_rng(seed)
    N = np.rint(np.exp(rng.uniform(math.log(N_min), math.log(N_max), size=n))).astype(np.int64)
    f = rng.integers(1, 7, size=n).astype(np.float64)
    E_a = rng.uniform(2.0, 10.0, size=n)
    gaps = rng.exponential(1.0, size=n)
    seeds = rng.integers(1, 2**31 - 1, size=n)
    return [dict(id=k, N=int(N[k]), f=float(f[k]), E_a=float(E_a[k]), rho=rho, steps=steps,
                 gap=float(gaps[k]), seed=int(seeds[k])) for k in range(n)]
