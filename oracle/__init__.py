"""FP64 CPU oracle for the valency-bounding correction (VBC), arXiv 2609.07842.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
(``paper_2609_07842_amd``) never imports it, and the two share no code.

The numerical work is in ``vbc_oracle.c`` (plain O(N^2) definitions in FP64,
built with ``-ffp-contract=off``); this module only builds that file with gcc
and marshals numpy arrays through ctypes.  Positions are N x 3 row-major here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vbc_oracle.c")
_LIB = os.path.join(_HERE, "libvbc_oracle.so")

PAIR_FIELDS = ("E_r", "r_r", "E_a", "r_a", "r_l", "r_h", "f", "delta")


class Pair(C.Structure):
    _fields_ = [(k, C.c_double) for k in PAIR_FIELDS]


def build(force: bool = True, out: str | None = None, extra_flags=()) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP), into `out` (default:
    next to the source) with optional extra flags (the sanitizer build of the tests)."""
    dst = out or _LIB
    if force or not os.path.exists(dst) or os.path.getmtime(dst) < os.path.getmtime(_SRC):
        tmp = dst + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               *extra_flags, "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, dst)
    return dst


_lib = None


def lib():
    global _lib
    if _lib is None:
        # VBC_ORACLE_LIBRARY: an already built copy (the tests' sanitizer build) instead
        path = os.environ.get("VBC_ORACLE_LIBRARY")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        pp = C.POINTER(Pair)
        for name in ("vbco_omega", "vbco_omega_d"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 3
        for name in ("vbco_Vr", "vbco_Vr_d_over_r"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 3
        for name in ("vbco_Va", "vbco_Va_d"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double] * 4
        L.vbco_neighbor_pairs.restype = C.c_int64
        L.vbco_neighbor_pairs.argtypes = [C.c_int64, dp, dp, C.c_double, i64p, C.c_int64]
        L.vbco_counts.restype = None
        L.vbco_counts.argtypes = [C.c_int64, dp, i32p, dp, C.c_int, pp, u32p, dp]
        L.vbco_eval.restype = None
        L.vbco_eval.argtypes = [C.c_int64, dp, i32p, dp, C.c_int, pp, u32p, dp, dp, dp, dp, dp]
        L.vbco_eval_subset.restype = None
        L.vbco_eval_subset.argtypes = [C.c_int64, dp, i32p, dp, C.c_int, pp, u32p, i64p,
                                       C.c_int64, dp, dp, dp]
        L.vbco_bonds.restype = C.c_double
        L.vbco_bonds.argtypes = [C.c_int64, dp, dp, i64p, C.c_int64, C.c_double, C.c_double, dp, dp]
        L.vbco_set_exclusions.restype = None
        L.vbco_set_exclusions.argtypes = [C.c_int64, C.c_int64]
        L.vbco_observables.restype = None
        L.vbco_observables.argtypes = [C.c_int64, dp, i32p, dp, C.c_int, pp, i32p, i32p]
        L.vbco_bond_clusters.restype = None
        L.vbco_bond_clusters.argtypes = [C.c_int64, dp, i32p, dp, C.c_int, pp, i64p, i32p]
        L.vbco_philox4x32_10.restype = None
        L.vbco_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.vbco_noise.restype = None
        L.vbco_noise.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, dp]
        L.vbco_run.restype = None
        L.vbco_run.argtypes = [C.c_int64, dp, dp, i32p, i64p, dp, C.c_int, pp, u32p, i64p,
                               C.c_int64, C.c_double, C.c_double, C.c_int, C.c_double,
                               C.c_double, C.c_double, C.c_uint64, C.c_uint64, C.c_int64,
                               dp, dp, dp]
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def pair_table(params, ntypes: int = 1):
    """params: dict (single type) or list of ntypes*ntypes dicts (row-major, symmetric)."""
    if isinstance(params, dict):
        params = [params]
    if len(params) != ntypes * ntypes:
        raise ValueError("need ntypes^2 pair entries")
    arr = (Pair * len(params))()
    for k, p in enumerate(params):
        for f in PAIR_FIELDS:
            setattr(arr[k], f, float(p[f]))
    return arr


def _sys_args(x, L, params, types, mask):
    x = _f64(x)
    N = x.shape[0]
    L = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy())
    if isinstance(params, dict):
        ntypes = 1
    else:
        ntypes = int(round(len(params) ** 0.5))
    tab = pair_table(params, ntypes)
    if types is not None:
        types = np.ascontiguousarray(types, dtype=np.int32)
        tp = types.ctypes.data_as(C.POINTER(C.c_int32))
    else:
        tp = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint32)
        mp = mask.ctypes.data_as(C.POINTER(C.c_uint32))
    else:
        mp = None
    return x, N, L, ntypes, tab, types, tp, mask, mp


# ---------------------------------------------------------------------------
# public wrappers
# ---------------------------------------------------------------------------

def omega(x, x1, x2):
    return lib().vbco_omega(float(x), float(x1), float(x2))


def omega_d(x, x1, x2):
    return lib().vbco_omega_d(float(x), float(x1), float(x2))


def V_r(r, E_r, r_r):
    return lib().vbco_Vr(float(r), float(E_r), float(r_r))


def V_r_d_over_r(r, E_r, r_r):
    return lib().vbco_Vr_d_over_r(float(r), float(E_r), float(r_r))


def V_a(r, E_a, r_r, r_a):
    return lib().vbco_Va(float(r), float(E_a), float(r_r), float(r_a))


def V_a_d(r, E_a, r_r, r_a):
    return lib().vbco_Va_d(float(r), float(E_a), float(r_r), float(r_a))


def neighbor_pairs(x, L, rc):
    """All pairs i<j with minimum-image r^2 < rc^2, lexicographic, shape (P, 2)."""
    x = _f64(x)
    Lv = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy())
    N = x.shape[0]
    cap = max(16, N * 8)
    while True:
        out = np.zeros((cap, 2), dtype=np.int64)
        n = lib().vbco_neighbor_pairs(N, _dp(x), _dp(Lv), float(rc),
                                      out.ctypes.data_as(C.POINTER(C.c_int64)), cap)
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


class _Exclusions:
    """Chain exclusions for the evaluations inside a with-block (none outside)."""

    def __init__(self, chain_len, excl_span):
        self.c, self.e = int(chain_len or 0), int(excl_span or 0)

    def __enter__(self):
        lib().vbco_set_exclusions(self.c, self.e)

    def __exit__(self, *a):
        lib().vbco_set_exclusions(0, 0)


def counts(x, L, params, types=None, mask=None, chain_len=0, excl_span=0):
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, mask)
    n = np.zeros(N)
    with _Exclusions(chain_len, excl_span):
        lib().vbco_counts(N, _dp(x), tp, _dp(Lv), nt, tab, mp, _dp(n))
    return n


def evaluate(x, L, params, types=None, mask=None, chain_len=0, excl_span=0):
    """Full evaluation.  Returns dict with n, A, F (N x 3), e, U, W, Wt (6).  With
    excl_span > 0, particles of one chain (chain_len consecutive indices) at most excl_span
    apart neither count each other nor attract."""
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, mask)
    n = np.zeros(N)
    A = np.zeros(N)
    F = np.zeros((N, 3))
    e = np.zeros(N)
    UW = np.zeros(8)
    with _Exclusions(chain_len, excl_span):
        lib().vbco_eval(N, _dp(x), tp, _dp(Lv), nt, tab, mp, _dp(n), _dp(A), _dp(F), _dp(e), _dp(UW))
    return {"n": n, "A": A, "F": F, "e": e, "U": UW[0], "W": UW[1], "Wt": UW[2:8].copy()}


def evaluate_subset(x, L, params, idx, types=None, mask=None, chain_len=0, excl_span=0):
    """n, F (m x 3) and e of the particles idx of a (possibly large) system."""
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, mask)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.shape[0]
    n = np.zeros(m)
    F = np.zeros((m, 3))
    e = np.zeros(m)
    with _Exclusions(chain_len, excl_span):
        lib().vbco_eval_subset(N, _dp(x), tp, _dp(Lv), nt, tab, mp,
                               idx.ctypes.data_as(C.POINTER(C.c_int64)), m, _dp(n), _dp(F), _dp(e))
    return {"n": n, "F": F, "e": e}


def bonds_energy_forces(x, L, bonds, k, r0, virial=False):
    """Energy and forces (N x 3) of harmonic bonds k/2 (r - r0)^2; with virial=True also
    the bonds' virial {W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz} (same convention as the
    pair virial of evaluate)."""
    x = _f64(x)
    N = x.shape[0]
    Lv = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy())
    b = np.ascontiguousarray(bonds, dtype=np.int64).reshape(-1, 2)
    F = np.zeros((N, 3))
    Wb = np.zeros(7)
    U = lib().vbco_bonds(N, _dp(x), _dp(Lv), b.ctypes.data_as(C.POINTER(C.c_int64)),
                         b.shape[0], float(k), float(r0), _dp(F), _dp(Wb))
    if virial:
        return U, F, Wb
    return U, F


def observables(x, L, params, types=None):
    """z_i (neighbours within r_a) and p_i (within r_r) of every particle, int32 arrays."""
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, None)
    z = np.zeros(N, dtype=np.int32)
    pen = np.zeros(N, dtype=np.int32)
    lib().vbco_observables(N, _dp(x), tp, _dp(Lv), nt, tab, z.ctypes.data_as(C.POINTER(C.c_int32)),
                           pen.ctypes.data_as(C.POINTER(C.c_int32)))
    return z, pen


def bond_clusters(x, L, params, types=None):
    """Connected components of the bond graph (r_ij < r_a of the pair, Section 3).

    Returns (label, z): label[i] is the smallest index of i's cluster (int64), z[i] the
    number of bonds of i (int32)."""
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, None)
    label = np.zeros(N, dtype=np.int64)
    z = np.zeros(N, dtype=np.int32)
    lib().vbco_bond_clusters(N, _dp(x), tp, _dp(Lv), nt, tab, label.ctypes.data_as(C.POINTER(C.c_int64)),
                             z.ctypes.data_as(C.POINTER(C.c_int32)))
    return label, z


def bond_clusters_large(x, L, params, types=None):
    """bond_clusters for systems too large for the O(N^2) loop, from library steps: candidate
    pairs within the largest r_a from a periodic k-d tree (scipy), the exact bond test of the
    plain definition on each candidate (t = x_i - x_j, d = t - L rint(t / L), r^2 = (dx dx +
    dy dy) + dz dz < r_a^2 of the pair, numpy elementwise FP64), and scipy's connected
    components.  Same (label, z) as bond_clusters; positions must lie in [0, L)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    N = len(x)
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    plist = [params] if isinstance(params, dict) else list(params)
    nt = int(round(len(plist) ** 0.5))
    ra = np.array([p["r_a"] for p in plist]).reshape(nt, nt)
    tp = np.zeros(N, dtype=np.int64) if types is None else np.asarray(types, dtype=np.int64)
    cand = cKDTree(x, boxsize=Lv).query_pairs(float(ra.max()) * (1.0 + 1e-9) + 1e-12, output_type="ndarray")
    i, j = cand[:, 0], cand[:, 1]
    t = x[i] - x[j]
    d = t - Lv * np.rint(t / Lv)
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    rr = ra[tp[i], tp[j]]
    keep = r2 < rr * rr
    i, j = i[keep], j[keep]
    z = (np.bincount(i, minlength=N) + np.bincount(j, minlength=N)).astype(np.int32)
    g = coo_matrix((np.ones(len(i), dtype=np.int8), (i, j)), shape=(N, N))
    nc, comp = connected_components(g, directed=False)
    first = np.full(nc, N, dtype=np.int64)
    np.minimum.at(first, comp, np.arange(N, dtype=np.int64))
    return first[comp], z


def bond_pairs(x, L, r_a):
    """Bonds of one snapshot (Section 3 criterion, r_ij < r_a, single type) as a set of
    index pairs (i, j), i < j, from the plain O(N^2) neighbour set."""
    ij = neighbor_pairs(x, L, r_a)
    return set(map(tuple, np.asarray(ij, dtype=np.int64).reshape(-1, 2).tolist()))


class BondTracker:
    """Bond lifetimes over a trajectory (Section 4): each bond is followed from the sample
    at which it is first seen to the first sample without it.  Lifetimes of completed bonds
    go to hist (bin = lifetime // bin_steps, the last bin holds the longer ones); bonds present
    at the reset have no birth and are counted as censored when they break.
    stats = [formed, broken with a lifetime, broken without one, 0 (no capacity limit),
    bonds summed over the samples]."""

    def __init__(self, hist_len, bin_steps):
        self.hist = np.zeros(hist_len, dtype=np.int64)
        self.bin_steps = int(bin_steps)
        self.stats = np.zeros(5, dtype=np.int64)
        self.birth = {}

    def reset(self, pairs):
        self.hist[:] = 0
        self.stats[:] = 0
        self.birth = {p: None for p in pairs}
        self.stats[4] += len(pairs)

    def sample(self, pairs, step):
        for p in list(self.birth):
            if p not in pairs:
                b = self.birth.pop(p)
                if b is None:
                    self.stats[2] += 1
                else:
                    self.stats[1] += 1
                    self.hist[min((step - b) // self.bin_steps, len(self.hist) - 1)] += 1
        for p in pairs:
            if p not in self.birth:
                self.birth[p] = step
                self.stats[0] += 1
        self.stats[4] += len(pairs)


def cluster_stats(label, z, hist_len=0):
    """Per-cluster sizes s and bond counts e (half the sum of z over the cluster); a cluster is
    cyclic when it carries a loop, e >= s (a tree has e = s - 1).

    Returns dict: clusters, largest, cyclic_particles (N_cyc), bonds, cyclic_clusters, and,
    for hist_len > 0, hist[2][hist_len]: row 0 counts all clusters by size, row 1 the acyclic
    ones; index s < hist_len holds size s, index 0 the clusters of size >= hist_len."""
    label = np.asarray(label, dtype=np.int64)
    z = np.asarray(z, dtype=np.int64)
    roots, inv = np.unique(label, return_inverse=True)
    size = np.bincount(inv)
    ends = np.bincount(inv, weights=z).astype(np.int64)
    assert (ends % 2 == 0).all()
    edges = ends // 2
    cyc = edges >= size
    out = dict(clusters=int(len(roots)), largest=int(size.max()) if len(size) else 0,
               cyclic_particles=int(size[cyc].sum()), bonds=int(edges.sum()),
               cyclic_clusters=int(cyc.sum()), sizes=size, edges=edges, roots=roots)
    if hist_len > 0:
        h = np.zeros((2, hist_len), dtype=np.int64)
        b = np.where(size < hist_len, size, 0)
        np.add.at(h[0], b, 1)
        np.add.at(h[1], b[~cyc], 1)
        out["hist"] = h
    return out


def flory_stockmayer(s, f, p, rho):
    """Number density of tree clusters of size s for valency f and saturation p, eq. (fs):
    rho w_s (1-p)^f [p (1-p)^(f-2)]^(s-1), w_s = f (fs-s)! / ((fs-2s+2)! s!); the factorials
    in log form (lgamma)."""
    from math import lgamma, log, exp
    s = int(s)
    if f * s - 2 * s + 2 < 0:
        return 0.0  # the reciprocal of a factorial of a negative integer vanishes
    lw = log(f) + lgamma(f * s - s + 1) - lgamma(f * s - 2 * s + 3) - lgamma(s + 1)
    if p <= 0.0:
        return rho * exp(lw) if s == 1 else 0.0
    lt = f * log(1.0 - p) + (s - 1) * (log(p) + (f - 2) * log(1.0 - p))
    return rho * exp(lw + lt)


def philox4x32_10(counter, key):
    c = (C.c_uint32 * 4)(*[int(v) for v in counter])
    k = (C.c_uint32 * 2)(*[int(v) for v in key])
    o = (C.c_uint32 * 4)()
    lib().vbco_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def noise(seed, tag, step):
    xi = np.zeros(3)
    lib().vbco_noise(int(seed), int(tag), int(step), _dp(xi))
    return xi


NVE, LANGEVIN = 0, 1


def run(x, v, L, params, nsteps, kind=NVE, dt=0.005, kT=1.0, gamma=0.1, seed=0, step0=0,
        types=None, mask=None, tags=None, bonds=None, k_bond=0.0, r0=1.0, history=False,
        chain_len=0, excl_span=0):
    """Integrate in place on copies; returns dict x, v, F (+ U, K histories)."""
    x, N, Lv, nt, tab, types, tp, mask, mp = _sys_args(x, L, params, types, mask)
    x = x.copy()
    v = _f64(v).copy()
    if tags is not None:
        tags = np.ascontiguousarray(tags, dtype=np.int64)
        tg = tags.ctypes.data_as(C.POINTER(C.c_int64))
    else:
        tg = None
    if bonds is not None:
        bonds = np.ascontiguousarray(bonds, dtype=np.int64).reshape(-1, 2)
        bp, nb = bonds.ctypes.data_as(C.POINTER(C.c_int64)), bonds.shape[0]
    else:
        bp, nb = None, 0
    F = np.zeros((N, 3))
    Uh = np.zeros(max(nsteps, 1)) if history else None
    Kh = np.zeros(max(nsteps, 1)) if history else None
    with _Exclusions(chain_len, excl_span):
        lib().vbco_run(N, _dp(x), _dp(v), tp, tg, _dp(Lv), nt, tab, mp, bp, nb, float(k_bond),
                       float(r0), int(kind), float(dt), float(kT), float(gamma), int(seed),
                       int(step0), int(nsteps), _dp(F), _dp(Uh), _dp(Kh))
    out = {"x": x, "v": v, "F": F}
    if history:
        out["U"] = Uh[:nsteps]
        out["K"] = Kh[:nsteps]
    return out
