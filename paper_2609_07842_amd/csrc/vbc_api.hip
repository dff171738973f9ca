// vbc_api.hip -- host side of libvbc: parameter validation, cell/brick layout, the pool
// allocator of the workspace and the order of kernel launches behind each C entry point
// (include/vbc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "arena.h"
#include "vbc_internal.h"

using namespace vbc;

namespace {

// Per-replica geometry and the automatic choices it implies.
struct RepPlan {
    RepDev R;
    int64_t slots = 0;
    double own_mean = 0, k_mean = 0, rho_cell = 0;
    int nh = 1, ncb = 1;
    int k_max_auto = 0, stage_cap_auto = 0;
};

// Fixed capacity of a workspace.
struct Caps {
    int32_t nrep = 0, ntypes_max = 1, any_chains = 0, any_excl = 0, any_mask = 0, bcap_max = 0, nh_max = 1, ncb_max = 1;
    int64_t ntot = 0, nslots = 0;
    int32_t nbrick = 0, ncell = 0;
};

struct Offsets {
    size_t reps, brick_rep, wl0, wl1, wl_n, cell_rank, brick_rank0, cstart0, cstart1, ccnt0, ccnt1, bcnt0, bcnt1,
        bfill, x0, x1, v, Fst, xref, tag, type, lcell, xs, vs, tags, types, lcells, src, inv,
        smap, wmap, stotal, nl, nn, nd, sA, wcnt, wlst, part, flags, step, stats, bevals, bentries,
        stamps, stamp_n, thermo, tpend;
    size_t bytes;
};

}  // namespace

struct vbc_handle_s {
    Launch P;               // capacity-wide launch shape (all bricks)
    Buffers B;
    vbc_options opt;
    bool pool = false;      // made by vbc_pool_create (admission checks list and staging)
    std::vector<RepDev> reps;   // host copy of every replica slot (n == 0: free)
    std::vector<char> live, has_state, need_full, fvalid;
    Arena a_slot, a_brick, a_cell, a_caller;
    RepDev *up = nullptr;       // pinned upload staging, one entry per slot
    std::vector<hipEvent_t> up_ev;
    std::vector<char> up_pending;
    int cur = 0;            // which position buffer holds the current positions
    std::string err;
    // kernel timing (vbc_profile)
    bool prof = false;
    int prof_max = 0;
    std::vector<hipEvent_t> ev[VBC_NK][2];
    int prof_n[VBC_NK] = {0, 0, 0, 0, 0, 0};
    // step time stamps (vbc_stamps)
    bool stamps = false;
    // energy and virial of every step accumulated per replica (vbc_thermo)
    bool thermo = false;
    // captured step graphs
    struct GraphEntry {
        int kind, nsteps, c;
        bool stamps, thermo;
        StepArgs st;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    bool use_graphs = true;
    ~vbc_handle_s()
    {
        for (int k = 0; k < VBC_NK; ++k)
            for (int e = 0; e < 2; ++e)
                for (hipEvent_t x : ev[k][e]) (void)hipEventDestroy(x);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (size_t r = 0; r < up_ev.size(); ++r) {
            if (up_pending[r]) (void)hipEventSynchronize(up_ev[r]);
            (void)hipEventDestroy(up_ev[r]);
        }
        if (up) (void)hipHostFree(up);
    }
};

// Mid-call steps per captured graph of a long call (even, so that a replay ends on the
// buffer it started from); calls of at most CALL_GRAPH_MAX steps are captured whole.
static constexpr int GRAPH_STEPS = 8;
static constexpr int CALL_GRAPH_MAX = 64;
static constexpr size_t GRAPH_CACHE = 16;

// Record the launch(es) of one kernel class between two events when timing is on.
template <class Fn>
static hipError_t timed(vbc_handle h, int kind, hipStream_t s, Fn &&fn)
{
    bool on = h->prof && h->prof_n[kind] < h->prof_max;
    if (!on) return fn();
    // the pass's own dispatches record the events (no marker packets around it)
    hipEvent_t e0 = h->ev[kind][0][h->prof_n[kind]], e1 = h->ev[kind][1][h->prof_n[kind]];
    set_launch_events(e0, e1);
    hipError_t e = fn();
    const int used = launch_events_used();
    if (e == hipSuccess) e = launch_events_error();
    set_launch_events(nullptr, nullptr);
    if (e != hipSuccess) return e;
    if (used == 0) {
        // nothing launched: an empty interval
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
    }
    if (e == hipSuccess) h->prof_n[kind]++;
    return e;
}

namespace {

// A roctx range around an entry point: rocprofv3 --marker-trace shows the library's calls
// beside its kernels; without a profiler attached the calls return at once.
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

thread_local std::string g_err;

vbc_status fail(vbc_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

vbc_status hfail(vbc_handle h, vbc_status st, const std::string &msg)
{
    if (h) h->err = msg;
    g_err = msg;
    return st;
}

bool pair_ok(const vbc_pair_params &p, std::string &why)
{
    auto fin = [](double v) { return std::isfinite(v); };
    if (!(fin(p.E_r) && fin(p.r_r) && fin(p.E_a) && fin(p.r_a) && fin(p.r_l) && fin(p.r_h) &&
          fin(p.f) && fin(p.delta))) {
        why = "non-finite pair parameter";
        return false;
    }
    if (p.E_r < 0 || p.E_a < 0) { why = "E_r and E_a must be >= 0"; return false; }
    if (!(p.r_r > 0 && p.r_a > p.r_r)) { why = "need 0 < r_r < r_a"; return false; }
    if (!(p.r_l > 0 && p.r_h > p.r_l)) { why = "need 0 < r_l < r_h"; return false; }
    return true;
}

bool same_pair(const vbc_pair_params &a, const vbc_pair_params &b)
{
    return a.E_r == b.E_r && a.r_r == b.r_r && a.E_a == b.E_a && a.r_a == b.r_a &&
           a.r_l == b.r_l && a.r_h == b.r_h && a.f == b.f && a.delta == b.delta;
}

PairDev derive(const vbc_pair_params &p)
{
    PairDev q;
    std::memset(&q, 0, sizeof(q));
    q.E_r = p.E_r;
    q.r_r = p.r_r;
    q.E_a = p.E_a;
    q.r_a = p.r_a;
    q.r_l = p.r_l;
    q.r_h = p.r_h;
    q.x1 = p.f - p.delta;
    q.x2 = q.x1 + 1.0;
    q.rr2 = p.r_r * p.r_r;
    q.ra2 = p.r_a * p.r_a;
    q.rl2 = p.r_l * p.r_l;
    q.rh2 = p.r_h * p.r_h;
    q.inv_rr2 = 1.0 / q.rr2;
    q.c_r = -4.0 * p.E_r / q.rr2;
    q.m = 0.5 * (p.r_a + p.r_r);
    double w = 0.5 * (p.r_a - p.r_r);
    q.inv_w = 1.0 / w;
    q.c_a = 4.0 * p.E_a / w;
    q.inv_dw = 1.0 / (p.r_h - p.r_l);
    q.c_c = -4.0 / (p.r_h - p.r_l);
    q.f = p.f;
    q.attract = p.E_a > 0.0;
    return q;
}

size_t carve(size_t &off, size_t bytes)
{
    size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

int brick_default(int precision) { return precision == VBC_FP64 ? 3 : 4; }

vbc_status check_options(const vbc_options *opt_in, vbc_options &opt)
{
    std::memset(&opt, 0, sizeof(opt));
    if (opt_in) opt = *opt_in;
    if (opt.precision != VBC_FP64 && opt.precision != VBC_FP32_MIXED)
        return fail(VBC_ERR_ARG, "precision must be VBC_FP64 or VBC_FP32_MIXED");
    if (opt.brick < 0 || opt.brick > MAX_BRICK) return fail(VBC_ERR_ARG, "brick must be 0..6");
    if (opt.block != 0 && (opt.block < 64 || opt.block > 1024 || opt.block % 64))
        return fail(VBC_ERR_ARG, "block must be a multiple of 64 in 64..1024");
    if (opt.k_max < 0 || opt.k_max > 65528) return fail(VBC_ERR_ARG, "k_max must be 0..65528");
    if (opt.stage_cap < 0 || opt.stage_cap > 65534)
        return fail(VBC_ERR_ARG, "stage_cap must be 0..65534");
    if (!(opt.rho_max >= 0.0) || !std::isfinite(opt.rho_max)) return fail(VBC_ERR_ARG, "rho_max must be >= 0");
    if (!opt.brick) opt.brick = brick_default(opt.precision);
    return VBC_OK;
}

int k_max_for(double k_mean) { return std::min(65528, round_up((int)std::ceil(k_mean * 1.6 + 24.0), CHUNK)); }
int stage_cap_for(double rho_cell, int nh)
{
    return std::min(65504, round_up((int)std::ceil(rho_cell * nh * 1.3 + 96.0), 32));
}

// Geometry of one replica: cells of edge >= the list radius, bricks of up to brick^3 cells,
// slots per brick, derived pair constants.
vbc_status plan_replica(const vbc_replica_desc &d, int brick_target, double rho_max, RepPlan &out)
{
    RepDev &R = out.R;
    std::memset(&R, 0, sizeof(R));
    if (d.n < 1) return fail(VBC_ERR_ARG, "n must be >= 1");
    if (d.n > (int64_t)1 << 30) return fail(VBC_ERR_ARG, "replica too large");
    if (d.ntypes < 1 || d.ntypes > MAXT) return fail(VBC_ERR_ARG, "ntypes must be 1..4");
    if (!d.params) return fail(VBC_ERR_ARG, "params is NULL");
    if (!(d.skin >= 0.0) || !std::isfinite(d.skin)) return fail(VBC_ERR_ARG, "skin must be >= 0");
    double rc = 0.0;
    for (int a = 0; a < d.ntypes; ++a)
        for (int c = 0; c < d.ntypes; ++c) {
            const vbc_pair_params &p = d.params[a * d.ntypes + c];
            std::string why;
            if (!pair_ok(p, why)) return fail(VBC_ERR_ARG, why);
            if (!same_pair(p, d.params[c * d.ntypes + a]))
                return fail(VBC_ERR_ARG, "pair table must be symmetric");
            rc = std::max(rc, std::max(p.r_r, std::max(p.r_a, p.r_h)));
            R.pair[a * MAXT + c] = derive(p);
        }
    for (int a = 0; a < d.ntypes; ++a) R.mask[a] = d.count_mask ? d.count_mask[a] : 0xFu;
    double rl = rc + d.skin;
    R.rc2 = rc * rc;
    R.rlist2 = rl * rl;
    R.disp2 = 0.25 * d.skin * d.skin;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        double L = d.L[a];
        if (!(L > 0.0) || !std::isfinite(L)) return fail(VBC_ERR_ARG, "box edges must be > 0");
        if (!(L > 2.0 * rl))
            return fail(VBC_ERR_BOX, "box edge " + std::to_string(L) +
                                         " must exceed twice the list radius " + std::to_string(rl));
        int nc = (int)std::min(std::floor(L / rl), 4096.0);
        // a cell must be at least the list radius even after rounding of x / h
        while (nc > 1 && L / nc < rl * (1.0 + 1e-9)) --nc;
        if (nc < 3) return fail(VBC_ERR_BOX, "fewer than 3 cells along an axis");
        if (nc > 1023) nc = 1023;
        R.nc[a] = nc;
        R.L[a] = L;
        R.h[a] = L / nc;
        R.bd[a] = std::max(1, std::min(brick_target, nc - 2));
        R.nb[a] = (nc + R.bd[a] - 1) / R.bd[a];
        ncell *= nc;
    }
    if (ncell > (int64_t)1 << 28) return fail(VBC_ERR_ARG, "too many cells");
    R.ncell = (int32_t)ncell;
    R.nbrick = R.nb[0] * R.nb[1] * R.nb[2];
    R.ntypes = d.ntypes;
    R.chain_len = d.chain_len > 1 ? d.chain_len : 0;
    if (R.chain_len) {
        if (d.n % R.chain_len) return fail(VBC_ERR_ARG, "n must be a multiple of chain_len");
        if (!(d.k_bond >= 0.0) || !(d.r0_bond >= 0.0)) return fail(VBC_ERR_ARG, "bad bond parameters");
        if (d.r0_bond >= 0.5 * std::min(d.L[0], std::min(d.L[1], d.L[2])))
            return fail(VBC_ERR_BOX, "bond length must be below half the box");
    }
    if (d.excl_span < 0) return fail(VBC_ERR_ARG, "excl_span must be >= 0");
    if (d.excl_span > 0 && !R.chain_len) return fail(VBC_ERR_ARG, "excl_span needs chains");
    R.excl_span = R.chain_len ? d.excl_span : 0;
    R.k_bond = d.k_bond;
    R.r0_bond = d.r0_bond;
    R.seed = d.seed;
    R.n = d.n;
    // slots per brick: the mean occupancy of a full brick with room for fluctuations
    out.ncb = R.bd[0] * R.bd[1] * R.bd[2];
    out.nh = (R.bd[0] + 2) * (R.bd[1] + 2) * (R.bd[2] + 2);
    double per_cell = (double)d.n / (double)ncell;
    out.own_mean = per_cell * out.ncb;
    R.bcap = (int32_t)std::min((int64_t)round_up((int)std::ceil(out.own_mean * 1.4 + 64.0), 64),
                               std::max<int64_t>(64, d.n));
    if ((int64_t)R.bcap * R.nbrick < d.n) R.bcap = (int32_t)((d.n + R.nbrick - 1) / R.nbrick);
    out.slots = (int64_t)R.nbrick * R.bcap;
    double vol = d.L[0] * d.L[1] * d.L[2];
    out.rho_cell = per_cell;
    out.k_mean = (double)d.n / vol * 4.18879020478639 * rl * rl * rl;
    out.k_max_auto = k_max_for(out.k_mean);
    out.stage_cap_auto = stage_cap_for(out.rho_cell, out.nh);
    if (rho_max > 0.0) {
        // hold local densities up to rho_max (clustering, phase separation) anywhere
        const double cell_vol = R.h[0] * R.h[1] * R.h[2];
        const double own_hold = rho_max * cell_vol * out.ncb;
        int bc = round_up((int)std::ceil(own_hold * 1.05 + 16.0), 64);
        R.bcap = (int32_t)std::max<int64_t>(R.bcap, std::min<int64_t>(bc, std::max<int64_t>(64, d.n)));
        out.slots = (int64_t)R.nbrick * R.bcap;
        out.stage_cap_auto = std::max(out.stage_cap_auto,
                                      std::min(65504, round_up((int)std::ceil(rho_max * cell_vol * out.nh * 1.05 + 32.0), 32)));
        double k_hold = rho_max * 4.18879020478639 * rl * rl * rl;
        out.k_max_auto = std::max(out.k_max_auto,
                                  std::min(65528, round_up((int)std::ceil(k_hold * 1.2 + 16.0), CHUNK)));
    }
    return VBC_OK;
}

// A count mask that leaves out a type present in the replica: only the general pair path
// applies masks, so such a replica needs it even with a single type.
bool partial_mask(const RepDev &R)
{
    const uint32_t all = (1u << R.ntypes) - 1u;
    for (int a = 0; a < R.ntypes; ++a)
        if ((R.mask[a] & all) != all) return true;
    return false;
}

// Workspace layout for a capacity; every array is 256-byte aligned.
Offsets layout(const Caps &C, int precision, int nchunk, int stage_cap)
{
    Offsets o;
    size_t off = 0;
    const int64_t S = C.nslots;
    const size_t nb = (size_t)C.nbrick, nc = (size_t)C.ncell, nr = (size_t)C.nrep;
    o.reps = carve(off, sizeof(RepDev) * nr);
    o.brick_rep = carve(off, sizeof(int32_t) * nb);
    o.wl0 = carve(off, sizeof(int32_t) * nb);
    o.wl1 = carve(off, sizeof(int32_t) * nb);
    o.wl_n = carve(off, sizeof(int32_t) * 2);
    o.cell_rank = carve(off, sizeof(int32_t) * nc);
    o.brick_rank0 = carve(off, sizeof(int32_t) * nb);
    o.cstart0 = carve(off, sizeof(int32_t) * nc);
    o.cstart1 = carve(off, sizeof(int32_t) * nc);
    o.ccnt0 = carve(off, sizeof(int32_t) * nc);
    o.ccnt1 = carve(off, sizeof(int32_t) * nc);
    o.bcnt0 = carve(off, sizeof(int32_t) * nb);
    o.bcnt1 = carve(off, sizeof(int32_t) * nb);
    o.bfill = carve(off, sizeof(int32_t) * nb);
    o.x0 = carve(off, sizeof(double) * 3 * S);
    o.x1 = carve(off, sizeof(double) * 3 * S);
    o.v = carve(off, sizeof(double) * 3 * S);
    o.Fst = carve(off, sizeof(double) * 3 * S);
    o.xref = carve(off, sizeof(double) * 3 * S);
    o.tag = carve(off, sizeof(int32_t) * S);
    o.type = carve(off, sizeof(int32_t) * S);
    o.lcell = carve(off, S);
    o.xs = carve(off, sizeof(double) * 3 * S);
    o.vs = carve(off, sizeof(double) * 3 * S);
    o.tags = carve(off, sizeof(int32_t) * S);
    o.types = carve(off, sizeof(int32_t) * S);
    o.lcells = carve(off, S);
    o.src = carve(off, sizeof(int32_t) * S);
    o.inv = carve(off, sizeof(int32_t) * C.ntot);
    o.smap = carve(off, sizeof(int32_t) * nb * stage_cap);
    o.wmap = carve(off, nb * stage_cap);
    o.stotal = carve(off, sizeof(int32_t) * nb);
    o.nl = carve(off, 16 * (size_t)nchunk * S);
    o.nn = carve(off, sizeof(uint16_t) * S);
    o.nd = carve(off, sizeof(double) * S);
    o.sA = carve(off, (precision == VBC_FP64 ? 16 : 8) * (size_t)S);
    o.wcnt = carve(off, sizeof(int32_t) * nb);
    o.wlst = carve(off, sizeof(uint16_t) * S);
    o.part = carve(off, sizeof(double) * 8 * nb);
    o.flags = carve(off, sizeof(uint32_t) * nr);
    o.step = carve(off, sizeof(uint64_t) * nr);
    o.stats = carve(off, sizeof(unsigned long long) * 4 * nr);
    o.bevals = carve(off, sizeof(unsigned long long) * nb);
    o.bentries = carve(off, sizeof(uint32_t) * nb);
    o.stamps = carve(off, sizeof(unsigned long long) * STAMP_CAP);
    o.stamp_n = carve(off, sizeof(unsigned long long));
    o.thermo = carve(off, sizeof(double) * THERMO_WORDS * nr);
    o.tpend = carve(off, sizeof(int32_t) * nr);
    o.bytes = off;
    return o;
}

// Bytes of the workspace that a replica occupies: its share of every per-slot, per-brick,
// per-cell, per-particle and per-replica array of the layout above.
size_t footprint_bytes(const RepPlan &rp, int precision, int nchunk, int stage_cap)
{
    size_t per_slot = 7 * 24 + 5 * 4 + 2 + 16 * (size_t)nchunk + 2 + 2 + 8 + (precision == VBC_FP64 ? 16 : 8);
    size_t per_brick = 4 * 8 + 5 * (size_t)stage_cap + 4 + 64 + 8 + 4;
    size_t per_cell = 5 * 4;
    return per_slot * (size_t)rp.slots + per_brick * (size_t)rp.R.nbrick +
           per_cell * (size_t)rp.R.ncell + 4 * (size_t)rp.R.n + sizeof(RepDev) + 4 + 8 + 32 +
           8 * THERMO_WORDS;
}

// Launch shape and LDS bounds for a capacity.
Launch launch_for(const Caps &C, const vbc_options &opt)
{
    Launch P;
    std::memset(&P, 0, sizeof(P));
    P.nrep = C.nrep;
    P.ntot = C.ntot;
    P.nslots = C.nslots;
    P.ncell_tot = C.ncell;
    P.nbrick_tot = C.nbrick;
    P.b_lo = 0;
    P.nb_launch = C.nbrick;
    // with one replica slot every live brick is in the range and a rebuild is all or
    // nothing, so the work lists would only add a launch per step
    P.list = C.nrep > 1 ? 0 : -1;
    P.k_max = opt.k_max;
    P.nchunk = opt.k_max / CHUNK;
    P.block = opt.block;
    P.stage_cap = opt.stage_cap;
    P.nh_max = C.nh_max;
    P.bcap_max = C.bcap_max;
    P.ncb_max = C.ncb_max;
    P.ntypes_max = C.ntypes_max;
    P.any_chains = C.any_chains;
    P.multi = (C.ntypes_max > 1 || C.any_excl || C.any_mask) ? 1 : 0;
    P.precision = opt.precision;
    return P;
}

Launch restrict_to(const Launch &P, const RepDev &R)
{
    Launch Q = P;
    Q.b_lo = R.b_off;
    Q.nb_launch = R.nbrick;
    Q.list = -1;
    return Q;
}

template <class T> T *at(void *base, size_t off) { return (T *)((char *)base + off); }

vbc_status hip_fail(vbc_handle h, hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    if (h) h->err = m;
    g_err = m;
    return VBC_ERR_HIP;
}

#define VBC_TRY(h, expr, where)                                  \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return hip_fail(h, _e, where);     \
    } while (0)

// The largest dynamic LDS request of any kernel at launch shape P must fit the device's
// per-workgroup limit (with room for the kernels' static LDS).
static vbc_status check_lds(vbc_handle h, const Launch &P)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
    int lds_max = 0;
    e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(h, e, "hipDeviceGetAttribute");
    size_t need = std::max(std::max(lds_bytes_nlist(P), lds_bytes_count(P)),
                           std::max(std::max(lds_bytes_embed(P), lds_bytes_force(P)),
                                    std::max(lds_bytes_sort(P), lds_bytes_bonds(P))));
    if (need + 2048 > (size_t)lds_max) {
        std::string m = "staging needs " + std::to_string(need) +
                        " bytes of LDS per workgroup; the device allows " + std::to_string(lds_max) +
                        " (lower brick, stage_cap or block)";
        return h ? hfail(h, VBC_ERR_CAPACITY, m) : fail(VBC_ERR_CAPACITY, m);
    }
    return VBC_OK;
}

// Validate the capacity against the device's LDS, make the handle, carve the workspace
// and clear it (synchronously on s).
vbc_status make_handle(const Caps &C, const vbc_options &opt, bool pool, void *d_ws,
                       size_t ws_bytes, hipStream_t s, vbc_handle *out)
{
    Launch P = launch_for(C, opt);
    Offsets o = layout(C, opt.precision, P.nchunk, P.stage_cap);
    if (!d_ws) return fail(VBC_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)d_ws) & 255) return fail(VBC_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < o.bytes)
        return fail(VBC_ERR_CAPACITY, "workspace too small: need " + std::to_string(o.bytes) + " bytes");
    {
        vbc_status st = check_lds(nullptr, P);
        if (st != VBC_OK) return st;
    }

    vbc_handle h = new (std::nothrow) vbc_handle_s;
    if (!h) return fail(VBC_ERR_ARG, "out of host memory");
    h->P = P;
    h->opt = opt;
    h->pool = pool;
    h->reps.assign(C.nrep, RepDev{});
    for (auto &R : h->reps) std::memset(&R, 0, sizeof(R));
    h->live.assign(C.nrep, 0);
    h->has_state.assign(C.nrep, 0);
    h->need_full.assign(C.nrep, 0);
    h->fvalid.assign(C.nrep, 0);
    h->up_pending.assign(C.nrep, 0);
    // a fixed single replica (not a pool): count and force take its descriptor as a kernel
    // argument (h->reps is sized once here, so the pointer stays valid)
    h->P.one = (!pool && C.nrep == 1) ? h->reps.data() : nullptr;
    h->a_slot.init(C.nslots);
    h->a_brick.init(C.nbrick);
    h->a_cell.init(C.ncell);
    h->a_caller.init(C.ntot);
    Buffers &B = h->B;
    B.reps = at<RepDev>(d_ws, o.reps);
    B.brick_rep = at<int32_t>(d_ws, o.brick_rep);
    B.wl[0] = at<int32_t>(d_ws, o.wl0);
    B.wl[1] = at<int32_t>(d_ws, o.wl1);
    B.wl_n = at<int32_t>(d_ws, o.wl_n);
    B.cell_rank = at<int32_t>(d_ws, o.cell_rank);
    B.brick_rank0 = at<int32_t>(d_ws, o.brick_rank0);
    B.cstart[0] = at<int32_t>(d_ws, o.cstart0);
    B.cstart[1] = at<int32_t>(d_ws, o.cstart1);
    B.ccnt[0] = at<int32_t>(d_ws, o.ccnt0);
    B.ccnt[1] = at<int32_t>(d_ws, o.ccnt1);
    B.bcnt[0] = at<int32_t>(d_ws, o.bcnt0);
    B.bcnt[1] = at<int32_t>(d_ws, o.bcnt1);
    B.bfill = at<int32_t>(d_ws, o.bfill);
    B.x[0] = at<double>(d_ws, o.x0);
    B.x[1] = at<double>(d_ws, o.x1);
    B.v = at<double>(d_ws, o.v);
    B.Fst = at<double>(d_ws, o.Fst);
    B.xref = at<double>(d_ws, o.xref);
    B.tag = at<int32_t>(d_ws, o.tag);
    B.type = at<int32_t>(d_ws, o.type);
    B.lcell = at<uint8_t>(d_ws, o.lcell);
    B.xs = at<double>(d_ws, o.xs);
    B.vs = at<double>(d_ws, o.vs);
    B.tags = at<int32_t>(d_ws, o.tags);
    B.types = at<int32_t>(d_ws, o.types);
    B.lcells = at<uint8_t>(d_ws, o.lcells);
    B.src = at<int32_t>(d_ws, o.src);
    B.inv = at<int32_t>(d_ws, o.inv);
    B.smap = at<int32_t>(d_ws, o.smap);
    B.wmap = at<uint8_t>(d_ws, o.wmap);
    B.stotal = at<int32_t>(d_ws, o.stotal);
    B.nl = at<uint4>(d_ws, o.nl);
    B.nn = at<uint16_t>(d_ws, o.nn);
    B.nd = at<double>(d_ws, o.nd);
    B.sA = at<void>(d_ws, o.sA);
    B.wcnt = at<int32_t>(d_ws, o.wcnt);
    B.wlst = at<uint16_t>(d_ws, o.wlst);
    B.part = at<double>(d_ws, o.part);
    B.flags = at<uint32_t>(d_ws, o.flags);
    B.step = at<uint64_t>(d_ws, o.step);
    B.stats = at<unsigned long long>(d_ws, o.stats);
    B.bevals = at<unsigned long long>(d_ws, o.bevals);
    B.bentries = at<uint32_t>(d_ws, o.bentries);
    B.stamps = at<unsigned long long>(d_ws, o.stamps);
    B.stamp_n = at<unsigned long long>(d_ws, o.stamp_n);
    B.thermo = at<double>(d_ws, o.thermo);
    B.tpend = at<int32_t>(d_ws, o.tpend);

    hipError_t e = hipHostMalloc((void **)&h->up, sizeof(RepDev) * std::max(C.nrep, 1), hipHostMallocDefault);
    if (e == hipSuccess) {
        h->up_ev.assign(C.nrep, nullptr);
        for (int r = 0; r < C.nrep && e == hipSuccess; ++r)
            e = hipEventCreateWithFlags(&h->up_ev[r], hipEventDisableTiming);
    }
    // every brick starts free (owner -1: all bytes 0xFF), everything else at zero
    if (e == hipSuccess) e = hipMemsetAsync(d_ws, 0, o.bytes, s);
    if (e == hipSuccess) e = hipMemsetAsync(B.brick_rep, 0xFF, sizeof(int32_t) * C.nbrick, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        vbc_status r = hip_fail(nullptr, e, "workspace set-up");
        delete h;
        return r;
    }
    *out = h;
    return VBC_OK;
}

// Place a planned replica in a free slot: take its ranges, upload its descriptor and
// write its tables (stream-ordered after all earlier work on s).
vbc_status place(vbc_handle h, const RepPlan &rp, hipStream_t s, int32_t *rep_out)
{
    int r = -1;
    for (int k = 0; k < h->P.nrep; ++k)
        if (!h->live[k]) { r = k; break; }
    if (r < 0) return hfail(h, VBC_ERR_CAPACITY, "no free replica slot");
    RepDev R = rp.R;
    int64_t p = h->a_slot.take(rp.slots);
    int64_t b = p < 0 ? -1 : h->a_brick.take(R.nbrick);
    int64_t c = b < 0 ? -1 : h->a_cell.take(R.ncell);
    int64_t o = c < 0 ? -1 : h->a_caller.take(R.n);
    if (o < 0) {
        if (c >= 0) h->a_cell.give(c, R.ncell);
        if (b >= 0) h->a_brick.give(b, R.nbrick);
        if (p >= 0) h->a_slot.give(p, rp.slots);
        const char *what = p < 0 ? "particle slots" : b < 0 ? "bricks" : c < 0 ? "cells" : "particles";
        return hfail(h, VBC_ERR_CAPACITY, std::string("no contiguous range of ") + what + " left");
    }
    R.p_off = p;
    R.b_off = (int32_t)b;
    R.c_off = (int32_t)c;
    R.o_off = o;
    if (h->up_pending[r]) VBC_TRY(h, hipEventSynchronize(h->up_ev[r]), "upload wait");
    h->up[r] = R;
    VBC_TRY(h, hipMemcpyAsync(h->B.reps + r, h->up + r, sizeof(RepDev), hipMemcpyHostToDevice, s),
            "descriptor upload");
    VBC_TRY(h, hipEventRecord(h->up_ev[r], s), "upload event");
    h->up_pending[r] = 1;
    VBC_TRY(h, launch_admit(h->B, r, std::max<int64_t>(R.nbrick, R.ncell), s), "admit");
    h->reps[r] = R;
    h->live[r] = 1;
    h->has_state[r] = 0;
    h->need_full[r] = 0;
    h->fvalid[r] = 0;
    *rep_out = r;
    return VBC_OK;
}

bool any_live(vbc_handle h)
{
    for (char l : h->live)
        if (l) return true;
    return false;
}

bool all_have_state(vbc_handle h)
{
    for (int r = 0; r < h->P.nrep; ++r)
        if (h->live[r] && !h->has_state[r]) return false;
    return true;
}

}  // namespace

#define VBC_NEED_STATE(h)                                                      \
    do {                                                                       \
        if (!any_live(h)) return hfail(h, VBC_ERR_STATE, "no live replica");   \
        if (!all_have_state(h)) return hfail(h, VBC_ERR_STATE, "no state set"); \
    } while (0)

// Replicas whose state was set from caller-order input get a full build (bin, sort,
// list) of their own bricks before anything reads their layout.
static vbc_status ensure_layout(vbc_handle h, hipStream_t s)
{
    for (int r = 0; r < h->P.nrep; ++r) {
        if (!h->live[r] || !h->need_full[r]) continue;
        const RepDev &R = h->reps[r];
        Launch Q = restrict_to(h->P, R);
        VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_full_build(h->B, Q, h->cur, r, R.n, s); }),
                "full build");
        VBC_TRY(h, launch_flags(h->B, r, 1, VBC_FLAG_REBUILD | FLAG_FULL, false, s), "flags");
        h->need_full[r] = 0;
        h->fvalid[r] = 0;
    }
    return VBC_OK;
}

#define VBC_LAYOUT(h, s)                          \
    do {                                          \
        vbc_status _st = ensure_layout(h, s);     \
        if (_st != VBC_OK) return _st;            \
    } while (0)

static StepArgs no_step()
{
    StepArgs st;
    std::memset(&st, 0, sizeof(st));
    return st;
}

// count, embed and force of the current positions into Fst (and the optional outputs),
// over the bricks that Q covers
static vbc_status eval_forces(vbc_handle h, const Launch &Q, bool thermo, const StepArgs &st,
                              double *d_F, double *d_e, hipStream_t s)
{
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, Q, h->cur, s); }), "rebuild");
    VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, Q, h->cur, nullptr, 0, true, s); }), "count");
    VBC_TRY(h, timed(h, VBC_K_EMBED, s, [&] { return launch_embed(h->B, Q, h->cur, s); }), "embed");
    VBC_TRY(h, timed(h, VBC_K_FORCE, s, [&] {
                return launch_force(h->B, Q, h->cur, MODE_EVAL, thermo, st, d_F, d_e, s);
            }),
            "force");
    return VBC_OK;
}

// Forces for the replicas that have none stored yet: all bricks at once when no live
// replica has them, else replica by replica so that the others are left untouched.
static vbc_status eval_missing(vbc_handle h, const StepArgs &st, hipStream_t s)
{
    int missing = 0, live = 0;
    for (int r = 0; r < h->P.nrep; ++r)
        if (h->live[r]) {
            ++live;
            if (!h->fvalid[r]) ++missing;
        }
    if (!missing) return VBC_OK;
    if (missing == live) {
        vbc_status st2 = eval_forces(h, h->P, false, st, nullptr, nullptr, s);
        if (st2 != VBC_OK) return st2;
    } else {
        for (int r = 0; r < h->P.nrep; ++r) {
            if (!h->live[r] || h->fvalid[r]) continue;
            vbc_status st2 = eval_forces(h, restrict_to(h->P, h->reps[r]), false, st, nullptr, nullptr, s);
            if (st2 != VBC_OK) return st2;
        }
    }
    for (int r = 0; r < h->P.nrep; ++r)
        if (h->live[r]) h->fvalid[r] = 1;
    return VBC_OK;
}

// One step after the opening kick, from position buffer c: list rebuild when due, count,
// dU/dn, force with the closing kick (MODE_MID: and the opening of the next step), and
// the step's time stamp when those are on.  The pair-evaluation statistic is sampled on
// the steps with k % STATS_EVERY == 0, k = the step's index inside the call.
static constexpr int STATS_EVERY = 8;
static hipError_t launch_step(vbc_handle h, int c, const StepArgs &st, Mode mode, int k, hipStream_t s)
{
    const bool stats = k % STATS_EVERY == 0;
    hipError_t e = timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, c, s); });
    if (e == hipSuccess)
        e = timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, c, nullptr, 1, stats, s); });
    if (e == hipSuccess) e = timed(h, VBC_K_EMBED, s, [&] { return launch_embed(h->B, h->P, c, s); });
    // with the sums on, the force pass leaves the step's per-brick energy and virial sums,
    // which the next step's count pass adds (the call's last step: launch_thermo_flush)
    StepArgs sa = st;
    sa.acc = h->thermo ? 1 : 0;
    if (e == hipSuccess)
        e = timed(h, VBC_K_FORCE, s, [&] {
            return launch_force(h->B, h->P, c, mode, h->thermo, sa, nullptr, nullptr, s);
        });
    if (e == hipSuccess && h->stamps) e = launch_stamp(h->B, s);
    return e;
}

// The energy and virial sums of a call's last step, added at the end of the call.
static hipError_t launch_thermo_flush(vbc_handle h, hipStream_t s)
{
    if (!h->thermo) return hipSuccess;
    return timed(h, VBC_K_REDUCE, s, [&] { return launch_thermo_acc(h->B, h->P, s); });
}

static hipError_t launch_kick(vbc_handle h, int c, const StepArgs &st, hipStream_t s)
{
    return timed(h, VBC_K_KICK, s, [&] { return launch_kick_drift(h->B, h->P, c, st, s); });
}

static bool same_step_args(const StepArgs &a, const StepArgs &b)
{
    return a.kind == b.kind && a.dt == b.dt && a.hdt == b.hdt && a.c1 == b.c1 && a.c2s == b.c2s &&
           a.seed == b.seed;
}

// Graph kinds: 0 = GRAPH_STEPS mid-call steps from buffer c; 1 = a whole call of nsteps
// steps (opening kick, nsteps - 1 mid-call steps, closing step) from buffer c.  Captured
// once per setting on a private stream and launched on the caller's stream; they hold
// kernel nodes only, every data-dependent choice (rebuild or not, which bricks are live)
// is taken on the GPU, so replicas may enter and leave between launches.
static hipError_t get_graph(vbc_handle h, int kind, int nsteps, int c, const StepArgs &st,
                            hipGraphExec_t *out)
{
    for (auto &g : h->graphs)
        if (g.kind == kind && g.nsteps == nsteps && g.c == c && g.stamps == h->stamps &&
            g.thermo == h->thermo && same_step_args(g.st, st)) {
            *out = g.exec;
            return hipSuccess;
        }
    hipError_t e = hipSuccess;
    if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    int cc = c;
    if (kind == 0) {
        for (int k = 0; k < GRAPH_STEPS && le == hipSuccess; ++k) {
            le = launch_step(h, cc, st, MODE_MID, k, h->cap_stream);
            cc ^= 1;
        }
    } else {
        le = launch_kick(h, cc, st, h->cap_stream);
        cc ^= 1;
        for (int k = 1; k < nsteps && le == hipSuccess; ++k) {
            le = launch_step(h, cc, st, MODE_MID, k - 1, h->cap_stream);
            cc ^= 1;
        }
        if (le == hipSuccess) le = launch_step(h, cc, st, MODE_LAST, nsteps - 1, h->cap_stream);
        if (le == hipSuccess) le = launch_thermo_flush(h, h->cap_stream);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap_stream, &g);
    if (le != hipSuccess) e = le;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    if (h->graphs.size() >= GRAPH_CACHE) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back({kind, nsteps, c, h->stamps, h->thermo, st, ex});
    *out = ex;
    return hipSuccess;
}

extern "C" {

vbc_status vbc_workspace_size(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt_in,
                              size_t *bytes);

// Capacity, options and plans of a fixed replica set (vbc_create).
static vbc_status plan_set(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt_in,
                           Caps &C, vbc_options &opt, std::vector<RepPlan> &plans)
{
    if (!reps || nrep < 1) return fail(VBC_ERR_ARG, "need at least one replica");
    if (nrep > MAX_REPLICAS) return fail(VBC_ERR_ARG, "at most 1024 replicas per handle");
    vbc_status st = check_options(opt_in, opt);
    if (st != VBC_OK) return st;
    plans.resize(nrep);
    double rho_cell_max = 0.0, k_mean_max = 0.0, own_mean_max = 0.0;
    C.nrep = nrep;
    for (int r = 0; r < nrep; ++r) {
        st = plan_replica(reps[r], opt.brick, opt.rho_max, plans[r]);
        if (st != VBC_OK) {
            g_err = "replica " + std::to_string(r) + ": " + g_err;
            return st;
        }
        const RepPlan &p = plans[r];
        C.ntot += p.R.n;
        C.nslots += p.slots;
        C.nbrick += p.R.nbrick;
        C.ncell += p.R.ncell;
        C.nh_max = std::max(C.nh_max, p.nh);
        C.ncb_max = std::max(C.ncb_max, p.ncb);
        C.bcap_max = std::max(C.bcap_max, (int)p.R.bcap);
        C.ntypes_max = std::max(C.ntypes_max, (int)p.R.ntypes);
        if (p.R.chain_len) C.any_chains = 1;
        if (p.R.excl_span) C.any_excl = 1;
        if (partial_mask(p.R)) C.any_mask = 1;
        rho_cell_max = std::max(rho_cell_max, p.rho_cell);
        own_mean_max = std::max(own_mean_max, p.own_mean);
        k_mean_max = std::max(k_mean_max, p.k_mean);
        if (C.nslots >= ((int64_t)1 << 31) - 1 || C.nbrick >= (1 << 30) || C.ncell >= (1 << 30))
            return fail(VBC_ERR_ARG, "more than 2^31 slots in total");
    }
    if (!opt.block) opt.block = std::max(128, std::min(512, round_up((int)std::ceil(own_mean_max), 64)));
    int k_auto = k_max_for(k_mean_max), s_auto = stage_cap_for(rho_cell_max, C.nh_max);
    for (const RepPlan &p : plans) {
        k_auto = std::max(k_auto, p.k_max_auto);
        s_auto = std::max(s_auto, p.stage_cap_auto);
    }
    opt.k_max = opt.k_max ? round_up(opt.k_max, CHUNK) : k_auto;
    if (!opt.stage_cap) opt.stage_cap = std::min(C.any_excl ? 32767 : 65504, s_auto);
    if (C.any_excl && opt.stage_cap > 32767)
        return fail(VBC_ERR_ARG, "with chain exclusions stage_cap must be <= 32767");
    return VBC_OK;
}

vbc_status vbc_workspace_size(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt_in,
                              size_t *bytes)
{
    if (!bytes) return fail(VBC_ERR_ARG, "bytes is NULL");
    Caps C;
    vbc_options opt;
    std::vector<RepPlan> plans;
    vbc_status st = plan_set(reps, nrep, opt_in, C, opt, plans);
    if (st != VBC_OK) return st;
    *bytes = layout(C, opt.precision, opt.k_max / CHUNK, opt.stage_cap).bytes;
    return VBC_OK;
}

vbc_status vbc_create(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt_in,
                      void *d_ws, size_t ws_bytes, hipStream_t s, vbc_handle *out)
{
    if (!out) return fail(VBC_ERR_ARG, "out is NULL");
    *out = nullptr;
    Caps C;
    vbc_options opt;
    std::vector<RepPlan> plans;
    vbc_status st = plan_set(reps, nrep, opt_in, C, opt, plans);
    if (st != VBC_OK) return st;
    vbc_handle h = nullptr;
    st = make_handle(C, opt, false, d_ws, ws_bytes, s, &h);
    if (st != VBC_OK) return st;
    // first fit on empty ranges: replica r lands at the prefix sums of the ones before it
    for (int r = 0; r < nrep; ++r) {
        int32_t got = -1;
        st = place(h, plans[r], s, &got);
        if (st != VBC_OK || got != r) {
            if (st == VBC_OK) st = hfail(h, VBC_ERR_CAPACITY, "replica placement");
            g_err = h->err;
            delete h;
            return st;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        vbc_status r = hip_fail(nullptr, e, "vbc_create upload");
        delete h;
        return r;
    }
    *out = h;
    return VBC_OK;
}

static vbc_status check_caps(const vbc_pool_caps *caps, const vbc_options &opt, Caps &C)
{
    if (!caps) return fail(VBC_ERR_ARG, "caps is NULL");
    if (caps->max_replicas < 1 || caps->max_replicas > MAX_REPLICAS)
        return fail(VBC_ERR_ARG, "max_replicas must be 1..1024");
    if (caps->max_types < 1 || caps->max_types > MAXT) return fail(VBC_ERR_ARG, "max_types must be 1..4");
    if (caps->max_particles < 1 || caps->max_slots < caps->max_particles)
        return fail(VBC_ERR_ARG, "need 1 <= max_particles <= max_slots");
    if (caps->max_slots >= ((int64_t)1 << 31) - 1) return fail(VBC_ERR_ARG, "max_slots must be < 2^31");
    if (caps->max_bricks < 1 || caps->max_cells < caps->max_bricks)
        return fail(VBC_ERR_ARG, "need 1 <= max_bricks <= max_cells");
    if (caps->max_bcap < 64) return fail(VBC_ERR_ARG, "max_bcap must be >= 64");
    if (opt.k_max <= 0 || opt.stage_cap <= 0)
        return fail(VBC_ERR_ARG, "a pool needs k_max and stage_cap set explicitly");
    C.nrep = caps->max_replicas;
    C.ntypes_max = caps->max_types;
    C.any_chains = caps->chains ? 1 : 0;
    C.any_excl = C.any_chains;  // replicas with chains may carry exclusions
    if (C.any_excl && opt.stage_cap > 32767)
        return fail(VBC_ERR_ARG, "a pool with chains needs stage_cap <= 32767");
    C.bcap_max = caps->max_bcap;
    C.nh_max = (opt.brick + 2) * (opt.brick + 2) * (opt.brick + 2);
    C.ncb_max = opt.brick * opt.brick * opt.brick;
    C.ntot = caps->max_particles;
    C.nslots = caps->max_slots;
    C.nbrick = caps->max_bricks;
    C.ncell = caps->max_cells;
    return VBC_OK;
}

static vbc_status pool_options(const vbc_options *opt_in, vbc_options &opt)
{
    vbc_status st = check_options(opt_in, opt);
    if (st != VBC_OK) return st;
    if (!opt.block) opt.block = 256;
    opt.k_max = round_up(opt.k_max, CHUNK);
    return VBC_OK;
}

vbc_status vbc_pool_workspace_size(const vbc_pool_caps *caps, const vbc_options *opt_in, size_t *bytes)
{
    if (!bytes) return fail(VBC_ERR_ARG, "bytes is NULL");
    vbc_options opt;
    vbc_status st = pool_options(opt_in, opt);
    if (st != VBC_OK) return st;
    Caps C;
    st = check_caps(caps, opt, C);
    if (st != VBC_OK) return st;
    *bytes = layout(C, opt.precision, opt.k_max / CHUNK, opt.stage_cap).bytes;
    return VBC_OK;
}

vbc_status vbc_pool_create(const vbc_pool_caps *caps, const vbc_options *opt_in, void *d_ws,
                           size_t ws_bytes, hipStream_t s, vbc_handle *out)
{
    if (!out) return fail(VBC_ERR_ARG, "out is NULL");
    *out = nullptr;
    vbc_options opt;
    vbc_status st = pool_options(opt_in, opt);
    if (st != VBC_OK) return st;
    Caps C;
    st = check_caps(caps, opt, C);
    if (st != VBC_OK) return st;
    return make_handle(C, opt, true, d_ws, ws_bytes, s, out);
}

vbc_status vbc_replica_footprint(const vbc_replica_desc *d, const vbc_options *opt_in, vbc_footprint *out)
{
    if (!d || !out) return fail(VBC_ERR_ARG, "NULL argument");
    vbc_options opt;
    vbc_status st = check_options(opt_in, opt);
    if (st != VBC_OK) return st;
    RepPlan rp;
    st = plan_replica(*d, opt.brick, opt.rho_max, rp);
    if (st != VBC_OK) return st;
    int k_max = opt.k_max ? round_up(opt.k_max, CHUNK) : rp.k_max_auto;
    int stage_cap = opt.stage_cap ? opt.stage_cap : rp.stage_cap_auto;
    out->slots = rp.slots;
    out->bricks = rp.R.nbrick;
    out->cells = rp.R.ncell;
    out->bcap = rp.R.bcap;
    out->k_max = rp.k_max_auto;
    out->stage_cap = rp.stage_cap_auto;
    out->brick = std::max(rp.R.bd[0], std::max(rp.R.bd[1], rp.R.bd[2]));
    out->bytes = footprint_bytes(rp, opt.precision, k_max / CHUNK, stage_cap);
    return VBC_OK;
}

vbc_status vbc_admit(vbc_handle h, const vbc_replica_desc *d, const double *d_x, const double *d_v,
                     const int32_t *d_type, uint64_t step0, hipStream_t s, int32_t *rep_out)
{
    Range range_("vbc_admit");
    if (!h || !d || !d_x || !rep_out) return fail(VBC_ERR_ARG, "NULL argument");
    *rep_out = -1;
    RepPlan rp;
    vbc_status st = plan_replica(*d, h->opt.brick, h->opt.rho_max, rp);
    if (st != VBC_OK) return hfail(h, st, g_err);
    const RepDev &R = rp.R;
    if (R.ntypes > h->P.ntypes_max) return hfail(h, VBC_ERR_CAPACITY, "more particle types than the pool allows");
    if (R.chain_len && !h->P.any_chains) return hfail(h, VBC_ERR_CAPACITY, "the pool was made without chains");
    if (partial_mask(R) && !h->P.multi)
        return hfail(h, VBC_ERR_CAPACITY,
                     "a count mask that leaves out a type needs a pool made with max_types > 1 or chains");
    if (R.bcap > h->P.bcap_max)
        return hfail(h, VBC_ERR_CAPACITY, "replica needs " + std::to_string(R.bcap) +
                                              " slots per brick; the pool has " + std::to_string(h->P.bcap_max));
    if (rp.nh > h->P.nh_max || rp.ncb > h->P.ncb_max)
        return hfail(h, VBC_ERR_CAPACITY, "brick larger than the pool's");
    if (h->pool && (rp.k_max_auto > h->P.k_max || rp.stage_cap_auto > h->P.stage_cap))
        return hfail(h, VBC_ERR_CAPACITY, "replica too dense for the pool: needs k_max " +
                                              std::to_string(rp.k_max_auto) + ", stage_cap " +
                                              std::to_string(rp.stage_cap_auto));
    int32_t r = -1;
    st = place(h, rp, s, &r);
    if (st != VBC_OK) return st;
    const RepDev &Rp = h->reps[r];
    VBC_TRY(h, launch_set_state(h->B, h->P, h->cur, r, Rp.n, d_x, d_v, d_type, 0, Rp.n, step0, s),
            "set_state");
    h->has_state[r] = 1;
    h->need_full[r] = 1;
    *rep_out = r;
    return VBC_OK;
}

vbc_status vbc_retire(vbc_handle h, int32_t rep, hipStream_t s)
{
    Range range_("vbc_retire");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (rep < 0 || rep >= h->P.nrep || !h->live[rep]) return hfail(h, VBC_ERR_ARG, "no such live replica");
    RepDev &R = h->reps[rep];
    VBC_TRY(h, launch_retire(h->B, rep, R.b_off, R.nbrick, s), "retire");
    h->a_slot.give(R.p_off, (int64_t)R.nbrick * R.bcap);
    h->a_brick.give(R.b_off, R.nbrick);
    h->a_cell.give(R.c_off, R.ncell);
    h->a_caller.give(R.o_off, R.n);
    std::memset(&R, 0, sizeof(R));
    h->live[rep] = 0;
    h->has_state[rep] = 0;
    h->need_full[rep] = 0;
    h->fvalid[rep] = 0;
    return VBC_OK;
}

vbc_status vbc_replica_info(vbc_handle h, int32_t rep, int64_t *n, int64_t *caller_offset)
{
    if (!h || !n || !caller_offset) return fail(VBC_ERR_ARG, "NULL argument");
    if (rep < 0 || rep >= h->P.nrep) return hfail(h, VBC_ERR_ARG, "replica index out of range");
    *n = h->live[rep] ? h->reps[rep].n : 0;
    *caller_offset = h->live[rep] ? h->reps[rep].o_off : 0;
    return VBC_OK;
}

vbc_status vbc_destroy(vbc_handle h)
{
    delete h;
    return VBC_OK;
}

const char *vbc_last_error(vbc_handle h)
{
    if (h && !h->err.empty()) return h->err.c_str();
    return g_err.c_str();
}

vbc_status vbc_get_options(vbc_handle h, vbc_options *out)
{
    if (!h || !out) return fail(VBC_ERR_ARG, "NULL argument");
    *out = h->opt;
    return VBC_OK;
}

vbc_status vbc_tune_set(vbc_handle h, const vbc_options *t)
{
    if (!h || !t) return fail(VBC_ERR_ARG, "NULL argument");
    if (t->precision != h->opt.precision) return hfail(h, VBC_ERR_ARG, "precision is fixed at creation");
    if ((t->k_max && round_up(t->k_max, CHUNK) != h->opt.k_max) || (t->brick && t->brick != h->opt.brick) ||
        (t->stage_cap && t->stage_cap != h->opt.stage_cap))
        return hfail(h, VBC_ERR_UNIMPLEMENTED,
                     "k_max, brick and stage_cap set the workspace layout: make a new handle to change them");
    if (t->block) {
        if (t->block < 64 || t->block > 1024 || t->block % 64)
            return hfail(h, VBC_ERR_ARG, "block must be a multiple of 64 in 64..1024");
        if (t->block != h->P.block) {
            Launch Q = h->P;
            Q.block = t->block;
            vbc_status st = check_lds(h, Q);
            if (st != VBC_OK) return st;
            h->P.block = t->block;
            h->opt.block = t->block;
            for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
            h->graphs.clear();
        }
    }
    return VBC_OK;
}

vbc_status vbc_set_state(vbc_handle h, int32_t rep, const double *d_x, const double *d_v,
                         const int32_t *d_type, uint64_t step0, hipStream_t s)
{
    Range range_("vbc_set_state");
    if (!h || !d_x) return fail(VBC_ERR_ARG, "NULL argument");
    if (rep >= h->P.nrep || (rep >= 0 && !h->live[rep])) return hfail(h, VBC_ERR_ARG, "no such live replica");
    for (int r = 0; r < h->P.nrep; ++r) {
        if (!h->live[r] || (rep >= 0 && r != rep)) continue;
        const RepDev &R = h->reps[r];
        int64_t off = rep < 0 ? R.o_off : 0, stride = rep < 0 ? h->P.ntot : R.n;
        VBC_TRY(h, launch_set_state(h->B, h->P, h->cur, r, R.n, d_x, d_v, d_type, off, stride, step0, s),
                "set_state");
        h->has_state[r] = 1;
        h->need_full[r] = 1;
        h->fvalid[r] = 0;
    }
    return VBC_OK;
}

vbc_status vbc_get_state(vbc_handle h, int32_t rep, double *d_x, double *d_v, hipStream_t s)
{
    Range range_("vbc_get_state");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (rep >= h->P.nrep || (rep >= 0 && !h->live[rep])) return hfail(h, VBC_ERR_ARG, "no such live replica");
    if (rep >= 0 ? !h->has_state[rep] : !all_have_state(h)) return hfail(h, VBC_ERR_STATE, "no state set");
    VBC_LAYOUT(h, s);
    for (int r = 0; r < h->P.nrep; ++r) {
        if (!h->live[r] || (rep >= 0 && r != rep)) continue;
        const RepDev &R = h->reps[r];
        int64_t off = rep < 0 ? R.o_off : 0, stride = rep < 0 ? h->P.ntot : R.n;
        VBC_TRY(h, launch_get_state(h->B, h->P, h->cur, r, (int64_t)R.nbrick * R.bcap, off, stride, d_x, d_v, s),
                "get_state");
    }
    return VBC_OK;
}

vbc_status vbc_build_nlist(vbc_handle h, hipStream_t s)
{
    Range range_("vbc_build_nlist");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_NEED_STATE(h);
    bool full = false;
    for (int r = 0; r < h->P.nrep; ++r) full = full || (h->live[r] && h->need_full[r]);
    VBC_LAYOUT(h, s);
    if (full) return VBC_OK;
    VBC_TRY(h, launch_flags(h->B, 0, h->P.nrep, VBC_FLAG_REBUILD, true, s), "flags");
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, launch_flags(h->B, 0, h->P.nrep, VBC_FLAG_REBUILD, false, s), "flags");
    for (int r = 0; r < h->P.nrep; ++r) h->fvalid[r] = 0;
    return VBC_OK;
}

vbc_status vbc_count(vbc_handle h, double *d_n, hipStream_t s)
{
    Range range_("vbc_count");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_NEED_STATE(h);
    VBC_LAYOUT(h, s);
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, h->cur, d_n, 0, true, s); }), "count");
    return VBC_OK;
}

vbc_status vbc_force(vbc_handle h, double *d_F, double *d_e, double *d_UW, hipStream_t s)
{
    Range range_("vbc_force");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_NEED_STATE(h);
    VBC_LAYOUT(h, s);
    bool thermo = d_e || d_UW;
    vbc_status st = eval_forces(h, h->P, thermo, no_step(), d_F, d_e, s);
    if (st != VBC_OK) return st;
    if (d_UW)
        VBC_TRY(h, timed(h, VBC_K_REDUCE, s, [&] { return launch_reduce(h->B, h->P, d_UW, s); }),
                "reduce");
    for (int r = 0; r < h->P.nrep; ++r) h->fvalid[r] = h->live[r];
    return VBC_OK;
}

static vbc_status check_integrator(vbc_handle h, int32_t nsteps, const vbc_integrator *it)
{
    if (nsteps < 0) return hfail(h, VBC_ERR_ARG, "nsteps must be >= 0");
    if (it->kind != VBC_NVE && it->kind != VBC_LANGEVIN) return hfail(h, VBC_ERR_ARG, "bad integrator kind");
    if (!(it->dt > 0.0) || !std::isfinite(it->dt)) return hfail(h, VBC_ERR_ARG, "dt must be > 0");
    if (it->kind == VBC_LANGEVIN && (!(it->gamma >= 0.0) || !(it->kT >= 0.0)))
        return hfail(h, VBC_ERR_ARG, "gamma and kT must be >= 0");
    return VBC_OK;
}

static StepArgs step_args(const vbc_integrator *it)
{
    StepArgs st = no_step();
    st.kind = it->kind;
    st.dt = it->dt;
    st.hdt = 0.5 * it->dt;
    // same expressions as the plain integrator: c1 = exp(-gamma dt), c2s = sqrt(1-c1^2) sqrt(kT)
    st.c1 = std::exp(-it->gamma * it->dt);
    st.c2s = std::sqrt(1.0 - st.c1 * st.c1) * std::sqrt(it->kT);
    st.seed = it->seed;
    return st;
}

vbc_status vbc_step_prepare(vbc_handle h, int32_t nsteps, const vbc_integrator *it)
{
    Range range_("vbc_step_prepare");
    if (!h || !it) return fail(VBC_ERR_ARG, "NULL argument");
    vbc_status r = check_integrator(h, nsteps, it);
    if (r != VBC_OK) return r;
    if (nsteps == 0 || !h->use_graphs || h->prof) return VBC_OK;
    const StepArgs st = step_args(it);
    hipGraphExec_t ge = nullptr;
    if (nsteps <= CALL_GRAPH_MAX) VBC_TRY(h, get_graph(h, 1, nsteps, h->cur, st, &ge), "call graph");
    else if (nsteps - 1 >= GRAPH_STEPS) VBC_TRY(h, get_graph(h, 0, GRAPH_STEPS, h->cur ^ 1, st, &ge), "step graph");
    return VBC_OK;
}

vbc_status vbc_step(vbc_handle h, int32_t nsteps, const vbc_integrator *it, hipStream_t s)
{
    Range range_("vbc_step");
    if (!h || !it) return fail(VBC_ERR_ARG, "NULL argument");
    VBC_NEED_STATE(h);
    {
        vbc_status r0 = check_integrator(h, nsteps, it);
        if (r0 != VBC_OK) return r0;
    }
    if (nsteps == 0) return VBC_OK;
    VBC_LAYOUT(h, s);
    const StepArgs st = step_args(it);
    vbc_status r = eval_missing(h, st, s);
    if (r != VBC_OK) return r;
    const bool graphs = h->use_graphs && !h->prof;
    if (graphs && nsteps <= CALL_GRAPH_MAX) {
        // the whole call as one graph launch
        hipGraphExec_t ge = nullptr;
        VBC_TRY(h, get_graph(h, 1, nsteps, h->cur, st, &ge), "call graph");
        VBC_TRY(h, hipGraphLaunch(ge, s), "graph launch");
        h->cur ^= nsteps & 1;
        return VBC_OK;
    }
    // opening half-kick and drift of the first step, from the stored forces
    VBC_TRY(h, launch_kick(h, h->cur, st, s), "kick");
    h->cur ^= 1;
    // nsteps - 1 mid-call steps: whole graphs, then single steps; kernel timing needs the
    // individual launches, so it bypasses the graphs
    int mid = nsteps - 1, k = 0;
    if (graphs && mid >= GRAPH_STEPS) {
        hipGraphExec_t ge = nullptr;
        VBC_TRY(h, get_graph(h, 0, GRAPH_STEPS, h->cur, st, &ge), "step graph");
        for (; mid >= GRAPH_STEPS; mid -= GRAPH_STEPS, k += GRAPH_STEPS)
            VBC_TRY(h, hipGraphLaunch(ge, s), "graph launch");
    }
    for (; mid > 0; --mid, ++k) {
        VBC_TRY(h, launch_step(h, h->cur, st, MODE_MID, k, s), "step");
        h->cur ^= 1;
    }
    // last step: closing half-kick only; its forces are kept for the next call
    VBC_TRY(h, launch_step(h, h->cur, st, MODE_LAST, k, s), "step");
    VBC_TRY(h, launch_thermo_flush(h, s), "energy and virial sums");
    return VBC_OK;
}

vbc_status vbc_check(vbc_handle h, hipStream_t s, uint32_t *flags_per_replica)
{
    Range range_("vbc_check");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    std::vector<uint32_t> f(h->P.nrep);
    VBC_TRY(h, hipMemcpy(f.data(), h->B.flags, sizeof(uint32_t) * h->P.nrep, hipMemcpyDeviceToHost),
            "flags readback");
    for (int r = 0; r < h->P.nrep; ++r)
        if (!h->live[r]) f[r] = 0;
    if (flags_per_replica)
        for (int r = 0; r < h->P.nrep; ++r) flags_per_replica[r] = f[r] & 0xFFu;
    vbc_status st = VBC_OK;
    for (int r = 0; r < h->P.nrep && st == VBC_OK; ++r) {
        if (f[r] & VBC_FLAG_NONFINITE) {
            st = VBC_ERR_NONFINITE;
            h->err = "replica " + std::to_string(r) + ": non-finite coordinates or forces";
        } else if (f[r] & VBC_FLAG_STAGE_OVERFLOW) {
            st = VBC_ERR_CAPACITY;
            h->err = "replica " + std::to_string(r) +
                     ": brick slot or staging capacity exceeded (raise stage_cap or lower brick)";
        } else if (f[r] & VBC_FLAG_LOST) {
            st = VBC_ERR_NONFINITE;
            h->err = "replica " + std::to_string(r) +
                     ": a particle moved more than one cell between list builds (unstable dynamics)";
        } else if (f[r] & VBC_FLAG_NLIST_OVERFLOW) {
            st = VBC_ERR_NLIST_OVERFLOW;
            h->err = "replica " + std::to_string(r) + ": neighbour list overflow (raise k_max)";
        }
    }
    uint32_t errs = VBC_FLAG_NONFINITE | VBC_FLAG_NLIST_OVERFLOW | VBC_FLAG_STAGE_OVERFLOW | VBC_FLAG_LOST;
    VBC_TRY(h, launch_flags(h->B, 0, h->P.nrep, errs, false, s), "flags");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    return st;
}

vbc_status vbc_get_nlist(vbc_handle h, int32_t rep, int32_t *d_pairs, int64_t cap, int64_t *d_count,
                         hipStream_t s)
{
    if (!h || !d_count || (cap > 0 && !d_pairs)) return fail(VBC_ERR_ARG, "NULL argument");
    if (rep < 0 || rep >= h->P.nrep || !h->live[rep]) return hfail(h, VBC_ERR_ARG, "no such live replica");
    if (!h->has_state[rep]) return hfail(h, VBC_ERR_STATE, "no state set");
    VBC_LAYOUT(h, s);
    VBC_TRY(h, launch_rebuild(h->B, restrict_to(h->P, h->reps[rep]), h->cur, s), "rebuild");
    VBC_TRY(h, launch_export_nlist(h->B, h->P, rep, h->reps[rep].nbrick, d_pairs, cap, d_count, s),
            "export");
    return VBC_OK;
}

vbc_status vbc_observables(vbc_handle h, int32_t *d_z, int32_t *d_pen, int64_t *d_sums, hipStream_t s)
{
    Range range_("vbc_observables");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_NEED_STATE(h);
    VBC_LAYOUT(h, s);
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, launch_observe(h->B, h->P, h->cur, d_z, d_pen, d_sums, s), "observables");
    return VBC_OK;
}

static size_t cluster_array_bytes(const Launch &P) { return ((size_t)P.nslots * sizeof(int32_t) + 255) & ~(size_t)255; }

vbc_status vbc_cluster_scratch_size(vbc_handle h, size_t *bytes)
{
    if (!h || !bytes) return fail(VBC_ERR_ARG, "NULL argument");
    *bytes = 5 * cluster_array_bytes(h->P);
    return VBC_OK;
}

vbc_status vbc_clusters(vbc_handle h, void *d_scratch, size_t scratch_bytes, int32_t *d_label,
                        int64_t *d_stats, int64_t *d_hist, int32_t hist_len, hipStream_t s)
{
    Range range_("vbc_clusters");
    if (!h || !d_scratch) return fail(VBC_ERR_ARG, "NULL argument");
    if (scratch_bytes < 5 * cluster_array_bytes(h->P))
        return hfail(h, VBC_ERR_ARG, "scratch too small: vbc_cluster_scratch_size gives the size");
    if (((uintptr_t)d_scratch & 255) != 0) return hfail(h, VBC_ERR_ARG, "scratch must be 256-byte aligned");
    if (d_hist && (hist_len < 1 || hist_len > (1 << 24) || 2 * (int64_t)h->P.nrep * hist_len > INT32_MAX))
        return hfail(h, VBC_ERR_ARG, "hist_len must be 1..2^24, and 2 x slots x hist_len below 2^31, when d_hist is given");
    VBC_NEED_STATE(h);
    VBC_LAYOUT(h, s);
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    const size_t a = cluster_array_bytes(h->P);
    char *base = (char *)d_scratch;
    ClusterWork W;
    W.parent = (int32_t *)(base);
    W.size = (int32_t *)(base + a);
    W.ends = (uint32_t *)(base + 2 * a);
    W.mintag = (int32_t *)(base + 3 * a);
    W.z = (int32_t *)(base + 4 * a);
    VBC_TRY(h, launch_clusters(h->B, h->P, h->cur, W, d_label, d_stats, d_hist, d_hist ? hist_len : 0, s), "clusters");
    return VBC_OK;
}

// Scratch of vbc_clusters_noalloc: one fixed array in every GPU's memory, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not device memory:
// kernels and copies get the device address from hipGetSymbolAddress, looked up once per
// device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[VBC_CLUSTERS_NOALLOC_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the first call on
// that device, with the device current).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

vbc_status vbc_clusters_noalloc(vbc_handle h, int32_t *d_label, int64_t *d_stats, int64_t *d_hist,
                                int32_t hist_len, hipStream_t s)
{
    Range range_("vbc_clusters_noalloc");
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    const size_t need = 5 * cluster_array_bytes(h->P);
    if (need > (size_t)VBC_CLUSTERS_NOALLOC_BYTES)
        return hfail(h, VBC_ERR_CAPACITY,
                     "cluster scratch of " + std::to_string(need) + " bytes exceeds the library's fixed " +
                         std::to_string((size_t)VBC_CLUSTERS_NOALLOC_BYTES) +
                         " bytes: use vbc_clusters with caller scratch");
    void *p = nullptr;
    VBC_TRY(h, scratch_address(&p), "hipGetSymbolAddress(scratch)");
    // every scratch array is rewritten by the analysis' first kernel before it is read
    return vbc_clusters(h, p, need, d_label, d_stats, d_hist, hist_len, s);
}

static size_t track_part(size_t b) { return (b + 255) & ~(size_t)255; }

vbc_status vbc_bond_track_size(vbc_handle h, int32_t max_partners, size_t *bytes)
{
    if (!h || !bytes) return fail(VBC_ERR_ARG, "NULL argument");
    if (max_partners < 1 || max_partners > 64) return hfail(h, VBC_ERR_ARG, "max_partners must be 1..64");
    const size_t n = (size_t)h->P.ntot;
    *bytes = track_part(n * 4) + track_part(n * max_partners * 4) + track_part(n * max_partners * 8);
    return VBC_OK;
}

vbc_status vbc_bond_track(vbc_handle h, void *d_state, size_t state_bytes, int32_t max_partners, int32_t reset,
                          int64_t *d_hist, int32_t hist_len, int64_t bin_steps, int64_t *d_stats, hipStream_t s)
{
    Range range_("vbc_bond_track");
    if (!h || !d_state) return fail(VBC_ERR_ARG, "NULL argument");
    size_t need = 0;
    vbc_status st = vbc_bond_track_size(h, max_partners, &need);
    if (st != VBC_OK) return st;
    if (state_bytes < need) return hfail(h, VBC_ERR_ARG, "tracker state too small: vbc_bond_track_size gives the size");
    if (((uintptr_t)d_state & 255) != 0) return hfail(h, VBC_ERR_ARG, "tracker state must be 256-byte aligned");
    if (d_hist && (hist_len < 1 || (int64_t)h->P.nrep * hist_len > INT32_MAX))
        return hfail(h, VBC_ERR_ARG, "hist_len must be >= 1, and slots x hist_len below 2^31, when d_hist is given");
    if (d_hist && bin_steps < 1) return hfail(h, VBC_ERR_ARG, "bin_steps must be >= 1");
    VBC_NEED_STATE(h);
    VBC_LAYOUT(h, s);
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    const size_t n = (size_t)h->P.ntot;
    char *base = (char *)d_state;
    BondTrack T;
    T.count = (int32_t *)base;
    T.tags = (int32_t *)(base + track_part(n * 4));
    T.births = (int64_t *)(base + track_part(n * 4) + track_part(n * max_partners * 4));
    T.M = max_partners;
    VBC_TRY(h, launch_bond_track(h->B, h->P, h->cur, T, reset ? 1 : 0, d_hist, d_hist ? hist_len : 0,
                                 bin_steps, d_stats, s),
            "bond tracker");
    return VBC_OK;
}

vbc_status vbc_get_stats(vbc_handle h, hipStream_t s, vbc_stats *out)
{
    if (!h || !out) return fail(VBC_ERR_ARG, "NULL argument");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    std::vector<unsigned long long> v(4 * (size_t)h->P.nrep), ev(h->P.nbrick_tot);
    std::vector<uint32_t> en(h->P.nbrick_tot);
    VBC_TRY(h, hipMemcpy(v.data(), h->B.stats, sizeof(unsigned long long) * v.size(),
                         hipMemcpyDeviceToHost),
            "stats readback");
    VBC_TRY(h, hipMemcpy(ev.data(), h->B.bevals, sizeof(unsigned long long) * ev.size(),
                         hipMemcpyDeviceToHost),
            "stats readback");
    VBC_TRY(h, hipMemcpy(en.data(), h->B.bentries, sizeof(uint32_t) * en.size(),
                         hipMemcpyDeviceToHost),
            "stats readback");
    for (int r = 0; r < h->P.nrep; ++r) {
        const RepDev &R = h->reps[r];
        unsigned long long pe = 0, le = 0;
        if (h->live[r])
            for (int b = 0; b < R.nbrick; ++b) {
                pe += ev[R.b_off + b];
                le += en[R.b_off + b];
            }
        out[r].builds = h->live[r] ? v[4 * r] : 0;
        out[r].list_entries = le;
        out[r].pair_evals = pe;
        out[r].evals = h->live[r] ? v[4 * r + 3] : 0;
    }
    return VBC_OK;
}

vbc_status vbc_profile(vbc_handle h, int32_t enable, int32_t max_launches)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (enable && max_launches <= 0) return hfail(h, VBC_ERR_ARG, "max_launches must be > 0");
    h->prof = enable != 0;
    for (int k = 0; k < VBC_NK; ++k) h->prof_n[k] = 0;
    if (!h->prof) return VBC_OK;
    h->prof_max = max_launches;
    for (int k = 0; k < VBC_NK; ++k)
        for (int e = 0; e < 2; ++e)
            while ((int)h->ev[k][e].size() < max_launches) {
                hipEvent_t x;
                VBC_TRY(h, hipEventCreate(&x), "hipEventCreate");
                h->ev[k][e].push_back(x);
            }
    return VBC_OK;
}

vbc_status vbc_profile_read(vbc_handle h, hipStream_t s, double *ms, int64_t *launches)
{
    if (!h || !ms || !launches) return fail(VBC_ERR_ARG, "NULL argument");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    for (int k = 0; k < VBC_NK; ++k) {
        double tot = 0.0;
        for (int i = 0; i < h->prof_n[k]; ++i) {
            float t = 0.0f;
            VBC_TRY(h, hipEventElapsedTime(&t, h->ev[k][0][i], h->ev[k][1][i]), "hipEventElapsedTime");
            tot += t;
        }
        ms[k] = tot;
        launches[k] = h->prof_n[k];
        h->prof_n[k] = 0;
    }
    return VBC_OK;
}

vbc_status vbc_thermo(vbc_handle h, int32_t enable, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if ((enable != 0) != h->thermo) {
        // the step graphs launch the force pass with or without the sums: recapture
        for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
        h->graphs.clear();
    }
    h->thermo = enable != 0;
    VBC_TRY(h, launch_thermo_clear(h->B, h->P.nrep, s), "thermo reset");
    return VBC_OK;
}

vbc_status vbc_thermo_read(vbc_handle h, hipStream_t s, double *out)
{
    if (!h || !out) return fail(VBC_ERR_ARG, "NULL argument");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    VBC_TRY(h, hipMemcpy(out, h->B.thermo, sizeof(double) * THERMO_WORDS * h->P.nrep, hipMemcpyDeviceToHost),
            "thermo readback");
    for (int r = 0; r < h->P.nrep; ++r)
        if (!h->live[r])
            for (int k = 0; k < THERMO_WORDS; ++k) out[(size_t)r * THERMO_WORDS + k] = 0.0;
    VBC_TRY(h, launch_thermo_clear(h->B, h->P.nrep, s), "thermo reset");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    return VBC_OK;
}

vbc_status vbc_stamps(vbc_handle h, int32_t enable, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    h->stamps = enable != 0;
    VBC_TRY(h, hipMemsetAsync(h->B.stamp_n, 0, sizeof(unsigned long long), s), "stamp reset");
    return VBC_OK;
}

vbc_status vbc_stamps_read(vbc_handle h, hipStream_t s, uint64_t *out, int64_t cap, int64_t *n,
                           double *hz)
{
    if (!h || !n || !hz || (cap > 0 && !out)) return fail(VBC_ERR_ARG, "NULL argument");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    unsigned long long total = 0;
    VBC_TRY(h, hipMemcpy(&total, h->B.stamp_n, sizeof(total), hipMemcpyDeviceToHost), "stamp count");
    int64_t keep = std::min<int64_t>((int64_t)total, std::min<int64_t>(STAMP_CAP, std::max<int64_t>(cap, 0)));
    std::vector<unsigned long long> ring(STAMP_CAP);
    if (keep > 0) {
        VBC_TRY(h, hipMemcpy(ring.data(), h->B.stamps, sizeof(unsigned long long) * STAMP_CAP,
                             hipMemcpyDeviceToHost),
                "stamp readback");
        for (int64_t k = 0; k < keep; ++k)
            out[k] = ring[(total - keep + (uint64_t)k) & (STAMP_CAP - 1)];
    }
    *n = keep;
    int dev = 0, khz = 0;
    VBC_TRY(h, hipGetDevice(&dev), "hipGetDevice");
    VBC_TRY(h, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "clock rate");
    *hz = 1e3 * (double)khz;
    VBC_TRY(h, hipMemsetAsync(h->B.stamp_n, 0, sizeof(unsigned long long), s), "stamp reset");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    return VBC_OK;
}

}  // extern "C"
