"""ctypes binding of libvbc.so (include/vbc.h) with the same entry-point names.

Only argument marshalling lives here: device memory comes from torch tensors, the
stream is torch's current stream, and every computation runs in the library's HIP
kernels.  Importing this module fails loudly if libvbc.so has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VBC_LIBRARY may name another build of the same library (side-by-side comparisons)
LIB_PATH = os.environ.get("VBC_LIBRARY") or os.path.join(_HERE, "libvbc.so")

VBC_OK, VBC_ERR_ARG, VBC_ERR_BOX, VBC_ERR_NLIST_OVERFLOW, VBC_ERR_NONFINITE, VBC_ERR_HIP, \
    VBC_ERR_CAPACITY, VBC_ERR_UNIMPLEMENTED, VBC_ERR_STATE = range(9)
STATUS_NAMES = {0: "VBC_OK", 1: "VBC_ERR_ARG", 2: "VBC_ERR_BOX", 3: "VBC_ERR_NLIST_OVERFLOW",
                4: "VBC_ERR_NONFINITE", 5: "VBC_ERR_HIP", 6: "VBC_ERR_CAPACITY",
                7: "VBC_ERR_UNIMPLEMENTED", 8: "VBC_ERR_STATE"}
FLAG_REBUILD, FLAG_NLIST_OVERFLOW, FLAG_STAGE_OVERFLOW, FLAG_NONFINITE, FLAG_LOST = 1, 2, 4, 8, 16
FP64, FP32_MIXED = 0, 1
NVE, LANGEVIN = 0, 1

# every symbol include/vbc.h declares
EXPORTS = ("vbc_workspace_size", "vbc_create", "vbc_destroy", "vbc_last_error", "vbc_set_state",
           "vbc_get_state", "vbc_build_nlist", "vbc_count", "vbc_force", "vbc_step", "vbc_check",
           "vbc_get_nlist", "vbc_get_options", "vbc_get_stats", "vbc_profile", "vbc_profile_read",
           "vbc_replica_footprint", "vbc_pool_workspace_size", "vbc_pool_create", "vbc_admit",
           "vbc_retire", "vbc_replica_info", "vbc_stamps", "vbc_stamps_read", "vbc_tune_set",
           "vbc_observables", "vbc_cluster_scratch_size", "vbc_clusters", "vbc_bond_track_size",
           "vbc_bond_track", "vbc_clusters_noalloc", "vbc_step_prepare", "vbc_thermo",
           "vbc_thermo_read")
KERNEL_CLASSES = ("build", "count", "embed", "force", "kick", "reduce")


class PairParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_r", "r_r", "E_a", "r_a", "r_l", "r_h", "f", "delta")]


class ReplicaDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("L", C.c_double * 3), ("ntypes", C.c_int32),
                ("params", C.POINTER(PairParams)), ("count_mask", C.POINTER(C.c_uint32)),
                ("skin", C.c_double), ("chain_len", C.c_int32), ("k_bond", C.c_double),
                ("r0_bond", C.c_double), ("seed", C.c_uint64), ("excl_span", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("k_max", C.c_int32), ("brick", C.c_int32),
                ("block", C.c_int32), ("stage_cap", C.c_int32), ("rho_max", C.c_double)]


class Integrator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dt", C.c_double), ("kT", C.c_double),
                ("gamma", C.c_double), ("seed", C.c_uint64)]


class PoolCaps(C.Structure):
    _fields_ = [("max_replicas", C.c_int32), ("max_types", C.c_int32), ("max_particles", C.c_int64),
                ("max_slots", C.c_int64), ("max_bricks", C.c_int32), ("max_cells", C.c_int32),
                ("max_bcap", C.c_int32), ("chains", C.c_int32)]


class Footprint(C.Structure):
    _fields_ = [("slots", C.c_int64), ("bricks", C.c_int32), ("cells", C.c_int32),
                ("bcap", C.c_int32), ("k_max", C.c_int32), ("stage_cap", C.c_int32),
                ("brick", C.c_int32), ("bytes", C.c_size_t)]


class Stats(C.Structure):
    _fields_ = [("builds", C.c_uint64), ("list_entries", C.c_uint64), ("pair_evals", C.c_uint64),
                ("evals", C.c_uint64)]


class VBCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2609_07842_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
        sig = {
            "vbc_workspace_size": [C.POINTER(ReplicaDesc), i32, C.POINTER(Options), C.POINTER(C.c_size_t)],
            "vbc_create": [C.POINTER(ReplicaDesc), i32, C.POINTER(Options), vp, C.c_size_t, vp,
                           C.POINTER(vp)],
            "vbc_destroy": [vp],
            "vbc_set_state": [vp, i32, dp, dp, dp, u64, vp],
            "vbc_get_state": [vp, i32, dp, dp, vp],
            "vbc_build_nlist": [vp, vp],
            "vbc_count": [vp, dp, vp],
            "vbc_force": [vp, dp, dp, dp, vp],
            "vbc_step": [vp, i32, C.POINTER(Integrator), vp],
            "vbc_check": [vp, vp, C.POINTER(C.c_uint32)],
            "vbc_get_nlist": [vp, i32, dp, i64, dp, vp],
            "vbc_get_options": [vp, C.POINTER(Options)],
            "vbc_get_stats": [vp, vp, C.POINTER(Stats)],
            "vbc_profile": [vp, i32, i32],
            "vbc_profile_read": [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
            "vbc_replica_footprint": [C.POINTER(ReplicaDesc), C.POINTER(Options), C.POINTER(Footprint)],
            "vbc_pool_workspace_size": [C.POINTER(PoolCaps), C.POINTER(Options), C.POINTER(C.c_size_t)],
            "vbc_pool_create": [C.POINTER(PoolCaps), C.POINTER(Options), vp, C.c_size_t, vp, C.POINTER(vp)],
            "vbc_admit": [vp, C.POINTER(ReplicaDesc), dp, dp, dp, u64, vp, C.POINTER(C.c_int32)],
            "vbc_retire": [vp, i32, vp],
            "vbc_replica_info": [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
            "vbc_stamps": [vp, i32, vp],
            "vbc_tune_set": [vp, C.POINTER(Options)],
            "vbc_observables": [vp, dp, dp, dp, vp],
            "vbc_cluster_scratch_size": [vp, C.POINTER(C.c_size_t)],
            "vbc_clusters": [vp, dp, C.c_size_t, dp, dp, dp, i32, vp],
            "vbc_clusters_noalloc": [vp, dp, dp, dp, i32, vp],
            "vbc_step_prepare": [vp, i32, C.POINTER(Integrator)],
            "vbc_thermo": [vp, i32, vp],
            "vbc_thermo_read": [vp, vp, C.POINTER(C.c_double)],
            "vbc_bond_track_size": [vp, i32, C.POINTER(C.c_size_t)],
            "vbc_bond_track": [vp, dp, C.c_size_t, i32, i32, dp, i32, i64, dp, vp],
            "vbc_stamps_read": [vp, vp, C.POINTER(C.c_uint64), i64, C.POINTER(C.c_int64),
                                C.POINTER(C.c_double)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int32
        L.vbc_last_error.argtypes = [vp]
        L.vbc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st, h=None):
    if st != VBC_OK:
        msg = lib().vbc_last_error(h)
        raise VBCError(st, msg.decode() if msg else "")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _pair_array(params, ntypes):
    if isinstance(params, dict):
        params = [params]
    if len(params) != ntypes * ntypes:
        raise ValueError("need ntypes^2 pair entries")
    arr = (PairParams * len(params))()
    for k, p in enumerate(params):
        for f in ("E_r", "r_r", "E_a", "r_a", "r_l", "r_h", "f", "delta"):
            setattr(arr[k], f, float(p[f]))
    return arr


def replica(n, L, params, mask=None, skin=0.4, chain_len=0, k_bond=0.0, r0_bond=1.0, seed=0,
            excl_span=0):
    """Description of one replica (host side).  params: dict or list of ntypes^2 dicts;
    seed is added to the integrator's seed to key this replica's noise; excl_span > 0
    (with chains) removes counting and attraction between beads of one chain at most that
    many beads apart."""
    ntypes = 1 if isinstance(params, dict) else int(round(len(params) ** 0.5))
    return dict(n=int(n), L=np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy(),
                params=params, ntypes=ntypes, mask=None if mask is None else np.asarray(mask, np.uint32),
                skin=float(skin), chain_len=int(chain_len), k_bond=float(k_bond), r0_bond=float(r0_bond),
                seed=int(seed), excl_span=int(excl_span))


def _descs(reps):
    arr = (ReplicaDesc * len(reps))()
    keep = []
    for k, r in enumerate(reps):
        pa = _pair_array(r["params"], r["ntypes"])
        keep.append(pa)
        d = arr[k]
        d.n = r["n"]
        for a in range(3):
            d.L[a] = float(r["L"][a])
        d.ntypes = r["ntypes"]
        d.params = C.cast(pa, C.POINTER(PairParams))
        if r["mask"] is not None:
            m = (C.c_uint32 * r["ntypes"])(*[int(v) for v in r["mask"]])
            keep.append(m)
            d.count_mask = C.cast(m, C.POINTER(C.c_uint32))
        else:
            d.count_mask = None
        d.skin = r["skin"]
        d.chain_len = r["chain_len"]
        d.k_bond = r["k_bond"]
        d.r0_bond = r["r0_bond"]
        d.seed = r.get("seed", 0) & 0xFFFFFFFFFFFFFFFF
        d.excl_span = int(r.get("excl_span", 0))
    return arr, keep


def _options(precision="fp64", k_max=0, brick=0, block=0, stage_cap=0, rho_max=0.0):
    o = Options()
    o.precision = FP64 if precision in ("fp64", FP64) else FP32_MIXED
    o.k_max, o.brick, o.block, o.stage_cap = int(k_max), int(brick), int(block), int(stage_cap)
    o.rho_max = float(rho_max)
    return o


def workspace_size(reps, precision="fp64", **opts):
    """Workspace bytes for a list of replica descriptions (host-only; no GPU needed)."""
    arr, keep = _descs(reps)
    o = _options(precision, **opts)
    n = C.c_size_t(0)
    st = lib().vbc_workspace_size(arr, len(reps), C.byref(o), C.byref(n))
    _check(st)
    return int(n.value)


def _soa(t, n, torch, device, dtype):
    """(n, 3) numpy/torch -> contiguous (3, n) device tensor."""
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device=device, dtype=dtype)
    if t.dim() == 2 and t.shape == (n, 3):
        t = t.t()
    return t.contiguous()


class _Handle:
    """Calls shared by a fixed replica set (System) and a pool (Pool)."""

    nslot = 0      # replica slots (reports and UW rows)
    stride = 0     # caller-order stride of per-particle arrays

    def _init_common(self, device):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.h = None

    def _alloc_ws(self, nbytes):
        self.ws_bytes = int(nbytes)
        self.ws = self.torch.empty(self.ws_bytes + 256, dtype=self.torch.uint8, device=self.device)
        self._ws_ptr = (self.ws.data_ptr() + 255) & ~255

    # -- plumbing -----------------------------------------------------------
    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _ok(self, st):
        _check(st, self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().vbc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def options(self):
        o = Options()
        self._ok(lib().vbc_get_options(self.h, C.byref(o)))
        return dict(precision=o.precision, k_max=o.k_max, brick=o.brick, block=o.block,
                    stage_cap=o.stage_cap, rho_max=o.rho_max)

    def tune_set(self, block=0):
        """Change the workgroup size of the brick kernels (layout knobs stay as created)."""
        o = Options()
        o.precision = self.options()["precision"]
        o.block = int(block)
        self._ok(lib().vbc_tune_set(self.h, C.byref(o)))

    def _n_of(self, rep):
        raise NotImplementedError

    # -- state --------------------------------------------------------------
    def _state_tensors(self, x, v, types, n):
        torch = self.torch
        xs = _soa(x, n, torch, self.device, torch.float64)
        vs = _soa(v, n, torch, self.device, torch.float64) if v is not None else None
        ts = None
        if types is not None:
            ts = (torch.from_numpy(np.ascontiguousarray(types)) if isinstance(types, np.ndarray)
                  else types).to(device=self.device, dtype=torch.int32).contiguous()
        return xs, vs, ts

    def set_state(self, x, v=None, types=None, rep=-1, step0=0):
        n = self.stride if rep < 0 else self._n_of(rep)
        xs, vs, ts = self._state_tensors(x, v, types, n)
        self._ok(lib().vbc_set_state(self.h, rep, _ptr(xs), _ptr(vs), _ptr(ts), int(step0),
                                     self._stream()))
        self._keep = (xs, vs, ts)  # alive until the copy kernel has run

    def get_state(self, rep=-1):
        torch = self.torch
        n = self.stride if rep < 0 else self._n_of(rep)
        x = torch.empty((3, n), dtype=torch.float64, device=self.device)
        v = torch.empty((3, n), dtype=torch.float64, device=self.device)
        self._ok(lib().vbc_get_state(self.h, rep, _ptr(x), _ptr(v), self._stream()))
        return x.t(), v.t()

    # -- the hot path -------------------------------------------------------
    def build_nlist(self):
        self._ok(lib().vbc_build_nlist(self.h, self._stream()))

    def count(self):
        n = self.torch.empty(self.stride, dtype=self.torch.float64, device=self.device)
        self._ok(lib().vbc_count(self.h, _ptr(n), self._stream()))
        return n

    def force(self, energies=True):
        torch = self.torch
        F = torch.empty((3, self.stride), dtype=torch.float64, device=self.device)
        e = torch.empty(self.stride, dtype=torch.float64, device=self.device) if energies else None
        UW = torch.empty((self.nslot, 8), dtype=torch.float64, device=self.device) if energies else None
        self._ok(lib().vbc_force(self.h, _ptr(F), _ptr(e), _ptr(UW), self._stream()))
        return F.t(), e, UW

    def observables(self):
        """z_i (neighbours within r_a), p_i (within r_r) as int32 tensors in caller order,
        and per replica {sum z, #(z > f), sum p} as an int64 tensor (slots, 3)."""
        torch = self.torch
        z = torch.empty(self.stride, dtype=torch.int32, device=self.device)
        p = torch.empty(self.stride, dtype=torch.int32, device=self.device)
        sums = torch.empty((self.nslot, 3), dtype=torch.int64, device=self.device)
        self._ok(lib().vbc_observables(self.h, _ptr(z), _ptr(p), _ptr(sums), self._stream()))
        return z, p, sums

    def clusters(self, hist_len=0, labels=True):
        """Clusters of the bond graph (r_ij < r_a): per particle the smallest tag of its
        cluster (int32, caller order, or None), per replica {clusters, largest, particles in
        cyclic clusters, bonds, cyclic clusters} (int64, (slots, 5)), and for hist_len > 0 the
        size histograms (int64, (slots, 2, hist_len): all clusters, acyclic clusters; bin 0
        holds the sizes >= hist_len)."""
        torch = self.torch
        nb = C.c_size_t()
        self._ok(lib().vbc_cluster_scratch_size(self.h, C.byref(nb)))
        # 256-byte aligned scratch carved from one byte tensor
        raw = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        scratch = raw[off:off + nb.value]
        lab = torch.empty(self.stride, dtype=torch.int32, device=self.device) if labels else None
        stats = torch.empty((self.nslot, 5), dtype=torch.int64, device=self.device)
        hist = torch.empty((self.nslot, 2, hist_len), dtype=torch.int64, device=self.device) if hist_len else None
        self._ok(lib().vbc_clusters(self.h, _ptr(scratch), nb.value, _ptr(lab), _ptr(stats), _ptr(hist),
                                    int(hist_len), self._stream()))
        return lab, stats, hist

    def clusters_noalloc(self, hist_len=0, labels=True):
        """As clusters(), with the library's own fixed scratch (vbc_clusters_noalloc)
        instead of a scratch tensor."""
        torch = self.torch
        lab = torch.empty(self.stride, dtype=torch.int32, device=self.device) if labels else None
        stats = torch.empty((self.nslot, 5), dtype=torch.int64, device=self.device)
        hist = torch.empty((self.nslot, 2, hist_len), dtype=torch.int64, device=self.device) if hist_len else None
        self._ok(lib().vbc_clusters_noalloc(self.h, _ptr(lab), _ptr(stats), _ptr(hist), int(hist_len),
                                            self._stream()))
        return lab, stats, hist

    def bond_tracker(self, max_partners=16, hist_len=4096, bin_steps=1):
        """A bond-lifetime tracker over this handle's replicas (reset at once from the
        current bonds); call .sample() after steps, read .hist (slots, hist_len) and .stats
        (slots, 5) as int64 tensors."""
        return BondTracker(self, max_partners, hist_len, bin_steps)

    @staticmethod
    def _integrator(integrator, dt, kT, gamma, seed):
        it = Integrator()
        it.kind = NVE if integrator in ("nve", NVE) else LANGEVIN
        it.dt, it.kT, it.gamma, it.seed = float(dt), float(kT), float(gamma), int(seed)
        return it

    def step(self, nsteps, integrator="nve", dt=0.005, kT=1.0, gamma=0.1, seed=0):
        it = self._integrator(integrator, dt, kT, gamma, seed)
        self._ok(lib().vbc_step(self.h, int(nsteps), C.byref(it), self._stream()))

    def prepare_step(self, nsteps, integrator="nve", dt=0.005, kT=1.0, gamma=0.1, seed=0):
        """Capture the step graphs a step() call with these arguments would launch next
        (vbc_step_prepare); launches nothing."""
        it = self._integrator(integrator, dt, kT, gamma, seed)
        self._ok(lib().vbc_step_prepare(self.h, int(nsteps), C.byref(it)))

    def thermo(self, enable=True):
        """Accumulate the energy and virial of every step (vbc_thermo); clears the sums."""
        self._ok(lib().vbc_thermo(self.h, 1 if enable else 0, self._stream()))

    def thermo_read(self):
        """Per replica slot: steps accumulated, the last step's {U, W, W_xx, W_yy, W_zz,
        W_xy, W_xz, W_yz} and their sums over those steps (then cleared)."""
        out = (C.c_double * (17 * self.nslot))()
        self._ok(lib().vbc_thermo_read(self.h, self._stream(), out))
        a = np.frombuffer(out, dtype=np.float64).reshape(self.nslot, 17).copy()
        return [dict(steps=int(r[0]), last=r[1:9].copy(), sum=r[9:17].copy()) for r in a]

    def check(self, raise_on_error=True):
        flags = (C.c_uint32 * self.nslot)()
        st = lib().vbc_check(self.h, self._stream(), flags)
        if raise_on_error:
            self._ok(st)
        return st, [int(f) for f in flags]

    def stats(self):
        out = (Stats * self.nslot)()
        self._ok(lib().vbc_get_stats(self.h, self._stream(), out))
        return [dict(builds=o.builds, list_entries=o.list_entries, pair_evals=o.pair_evals,
                     evals=o.evals) for o in out]

    def profile(self, enable=True, max_launches=4096):
        self._ok(lib().vbc_profile(self.h, 1 if enable else 0, int(max_launches) if enable else 0))

    def profile_read(self):
        ms = (C.c_double * 6)()
        n = (C.c_int64 * 6)()
        self._ok(lib().vbc_profile_read(self.h, self._stream(), ms, n))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def stamps(self, enable=True):
        self._ok(lib().vbc_stamps(self.h, 1 if enable else 0, self._stream()))

    def stamps_read(self, cap=1 << 16):
        """Device clock at the end of each stamped step since the last read (seconds)."""
        buf = (C.c_uint64 * cap)()
        n = C.c_int64(0)
        hz = C.c_double(0.0)
        self._ok(lib().vbc_stamps_read(self.h, self._stream(), buf, int(cap), C.byref(n), C.byref(hz)))
        return np.array(buf[: n.value], dtype=np.float64) / hz.value

    def nlist_pairs(self, rep=0, cap=None):
        torch = self.torch
        n = self._n_of(rep)
        if cap is None:
            cap = n * self.options()["k_max"]
        pairs = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=self.device)
        self._ok(lib().vbc_get_nlist(self.h, rep, _ptr(pairs), int(cap), _ptr(cnt), self._stream()))
        c = int(cnt.item())
        return pairs[: min(c, cap)].cpu().numpy(), c


class BondTracker:
    """State of vbc_bond_track for one handle (see include/vbc.h)."""

    def __init__(self, handle, max_partners, hist_len, bin_steps):
        torch = handle.torch
        self.h = handle
        self.M, self.hist_len, self.bin_steps = int(max_partners), int(hist_len), int(bin_steps)
        nb = C.c_size_t()
        handle._ok(lib().vbc_bond_track_size(handle.h, self.M, C.byref(nb)))
        self._raw = torch.empty(nb.value + 256, dtype=torch.uint8, device=handle.device)
        off = (-self._raw.data_ptr()) % 256
        self.state = self._raw[off:off + nb.value]
        self.hist = torch.empty((handle.nslot, self.hist_len), dtype=torch.int64, device=handle.device)
        self.stats = torch.empty((handle.nslot, 5), dtype=torch.int64, device=handle.device)
        self.sample(reset=True)

    def sample(self, reset=False):
        h = self.h
        h._ok(lib().vbc_bond_track(h.h, _ptr(self.state), self.state.numel(), self.M, 1 if reset else 0,
                                   _ptr(self.hist), self.hist_len, self.bin_steps, _ptr(self.stats), h._stream()))

    def median_lifetime(self, rep=0):
        """Median completed lifetime in steps, as the lower edge of its bin (exact when the
        samples are bin_steps apart), or None without any completed bond."""
        h = self.hist[rep].cpu().numpy()
        tot = int(h.sum())
        if tot == 0:
            return None
        k = int((h.cumsum() >= (tot + 1) // 2).argmax())
        return float(k * self.bin_steps)


class System(_Handle):
    """One or more replicas resident on one GPU behind a libvbc handle (vbc_create)."""

    def __init__(self, reps, precision="fp64", k_max=0, brick=0, block=0, stage_cap=0,
                 rho_max=0.0, device="cuda"):
        self._init_common(device)
        if isinstance(reps, dict):
            reps = [reps]
        self.reps = reps
        self.nrep = self.nslot = len(reps)
        self.ntot = self.stride = sum(r["n"] for r in reps)
        self.offsets = np.concatenate([[0], np.cumsum([r["n"] for r in reps])]).astype(np.int64)
        arr, keep = _descs(reps)
        o = _options(precision, k_max, brick, block, stage_cap, rho_max)
        n = C.c_size_t(0)
        _check(lib().vbc_workspace_size(arr, self.nrep, C.byref(o), C.byref(n)))
        self._alloc_ws(n.value)
        h = C.c_void_p()
        _check(lib().vbc_create(arr, self.nrep, C.byref(o), C.c_void_p(self._ws_ptr),
                                C.c_size_t(self.ws_bytes), self._stream(), C.byref(h)))
        self.h = h
        self.precision = precision

    def _n_of(self, rep):
        return self.reps[rep]["n"]


def footprint(rep, precision="fp64", **opts):
    """Layout of one replica and the workspace bytes it takes (host-only; no GPU needed)."""
    arr, keep = _descs([rep])
    o = _options(precision, **opts)
    fp = Footprint()
    _check(lib().vbc_replica_footprint(arr, C.byref(o), C.byref(fp)))
    return dict(slots=int(fp.slots), bricks=int(fp.bricks), cells=int(fp.cells), bcap=int(fp.bcap),
                k_max=int(fp.k_max), stage_cap=int(fp.stage_cap), brick=int(fp.brick),
                bytes=int(fp.bytes))


def _caps(max_replicas, max_particles, max_slots, max_bricks, max_cells, max_bcap, max_types, chains):
    c = PoolCaps()
    c.max_replicas, c.max_types = int(max_replicas), int(max_types)
    c.max_particles, c.max_slots = int(max_particles), int(max_slots)
    c.max_bricks, c.max_cells, c.max_bcap = int(max_bricks), int(max_cells), int(max_bcap)
    c.chains = 1 if chains else 0
    return c


def pool_workspace_size(caps, precision="fp32", **opts):
    c = _caps(**caps)
    o = _options(precision, **opts)
    n = C.c_size_t(0)
    _check(lib().vbc_pool_workspace_size(C.byref(c), C.byref(o), C.byref(n)))
    return int(n.value)


class Pool(_Handle):
    """A fixed-capacity pool of replicas that enter (admit) and leave (retire) while the
    others keep running (vbc_pool_create)."""

    def __init__(self, caps, precision="fp32", k_max=0, stage_cap=0, brick=0, block=0,
                 rho_max=0.0, device="cuda"):
        self._init_common(device)
        self.caps = dict(caps)
        c = _caps(**caps)
        self.nslot = c.max_replicas
        self.stride = c.max_particles
        o = _options(precision, k_max, brick, block, stage_cap, rho_max)
        n = C.c_size_t(0)
        _check(lib().vbc_pool_workspace_size(C.byref(c), C.byref(o), C.byref(n)))
        self._alloc_ws(n.value)
        h = C.c_void_p()
        _check(lib().vbc_pool_create(C.byref(c), C.byref(o), C.c_void_p(self._ws_ptr),
                                     C.c_size_t(self.ws_bytes), self._stream(), C.byref(h)))
        self.h = h
        self.precision = precision
        self._keep_admit = {}

    def _n_of(self, rep):
        return self.info(rep)[0]

    def info(self, rep):
        n, off = C.c_int64(0), C.c_int64(0)
        self._ok(lib().vbc_replica_info(self.h, int(rep), C.byref(n), C.byref(off)))
        return int(n.value), int(off.value)

    def admit(self, rep, x, v=None, types=None, step0=0):
        """Admit one replica (description from replica()) with its state; returns its slot."""
        arr, keep = _descs([rep])
        xs, vs, ts = self._state_tensors(x, v, types, rep["n"])
        r = C.c_int32(-1)
        self._ok(lib().vbc_admit(self.h, arr, _ptr(xs), _ptr(vs), _ptr(ts), int(step0),
                                 self._stream(), C.byref(r)))
        self._keep_admit[int(r.value)] = (xs, vs, ts)  # alive until the copy kernel has run
        return int(r.value)

    def retire(self, rep):
        self._ok(lib().vbc_retire(self.h, int(rep), self._stream()))
        self._keep_admit.pop(int(rep), None)
