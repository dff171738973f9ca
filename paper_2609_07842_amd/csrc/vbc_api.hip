// vbc_api.hip -- host side of libvbc: parameter validation, cell/brick layout, workspace
// carving and the order of kernel launches behind each C entry point (include/vbc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vbc_internal.h"

using namespace vbc;

struct vbc_handle_s {
    Launch P;
    Buffers B;
    std::vector<RepDev> reps;
    vbc_options opt;
    int cur = 0;            // which position buffer holds the current positions
    bool f_valid = false;   // Fst holds the forces of the current positions
    bool have_state = false;
    bool need_full = false; // unsorted input waiting for a full build
    std::string err;
    // kernel timing (vbc_profile)
    bool prof = false;
    int prof_max = 0;
    std::vector<hipEvent_t> ev[VBC_NK][2];
    int prof_n[VBC_NK] = {0, 0, 0, 0, 0, 0};
    // captured step graphs: GRAPH_STEPS mid-call steps starting from position buffer c
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    StepArgs gst[2];
    bool use_graphs = true;
    ~vbc_handle_s()
    {
        for (int k = 0; k < VBC_NK; ++k)
            for (int e = 0; e < 2; ++e)
                for (hipEvent_t x : ev[k][e]) (void)hipEventDestroy(x);
        for (int c = 0; c < 2; ++c)
            if (gexec[c]) (void)hipGraphExecDestroy(gexec[c]);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

// Steps per captured graph (even, so that a replay ends on the buffer it started from).
static constexpr int GRAPH_STEPS = 8;

// Record the launch(es) of one kernel class between two events when timing is on.
template <class Fn>
static hipError_t timed(vbc_handle h, int kind, hipStream_t s, Fn &&fn)
{
    bool on = h->prof && h->prof_n[kind] < h->prof_max;
    if (on) {
        hipError_t e = hipEventRecord(h->ev[kind][0][h->prof_n[kind]], s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = fn();
    if (e != hipSuccess) return e;
    if (on) {
        e = hipEventRecord(h->ev[kind][1][h->prof_n[kind]], s);
        h->prof_n[kind]++;
    }
    return e;
}

namespace {

thread_local std::string g_err;

struct Layout {
    Launch P;
    std::vector<RepDev> reps;
    std::vector<int32_t> cell_rank, brick_rank0;
    vbc_options opt;
    size_t bytes = 0;
    // byte offsets into the workspace
    size_t o_reps, o_cell_rank, o_brick_rank0, o_cstart0, o_cstart1, o_ccnt0, o_ccnt1, o_bcnt0,
        o_bcnt1, o_bfill, o_x0, o_x1, o_v, o_Fst, o_xref, o_tag, o_type, o_lcell, o_xs, o_vs,
        o_tags, o_types, o_lcells, o_src, o_inv, o_smap, o_wmap, o_stotal, o_nl, o_nn, o_nd, o_sA, o_win, o_part, o_flags,
        o_step, o_stats, o_bevals, o_bentries;
};

vbc_status fail(vbc_status st, const std::string &msg)
{
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

vbc_status plan(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt_in, Layout &Lo)
{
    if (!reps || nrep < 1) return fail(VBC_ERR_ARG, "need at least one replica");
    vbc_options opt;
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

    Launch &P = Lo.P;
    std::memset(&P, 0, sizeof(P));
    P.nrep = nrep;
    P.precision = opt.precision;
    int brick_target = opt.brick ? opt.brick : (opt.precision == VBC_FP64 ? 3 : 4);
    double rho_cell_max = 0.0, k_mean_max = 0.0, own_mean_max = 0.0;
    int64_t p_off = 0, o_off = 0;
    int32_t c_off = 0, b_off = 0;
    int nh_max = 1, ntypes_max = 1, any_chains = 0, bcap_max = 0, ncb_max = 1;
    Lo.reps.resize(nrep);
    for (int r = 0; r < nrep; ++r) {
        const vbc_replica_desc &d = reps[r];
        RepDev R;
        std::memset(&R, 0, sizeof(R));
        if (d.n < 1) return fail(VBC_ERR_ARG, "replica " + std::to_string(r) + ": n must be >= 1");
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
        for (int a = 0; a < d.ntypes; ++a)
            R.mask[a] = d.count_mask ? d.count_mask[a] : 0xFu;
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
            int nc = (int)std::floor(L / rl);
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
            any_chains = 1;
        }
        R.k_bond = d.k_bond;
        R.r0_bond = d.r0_bond;
        // slots per brick: the mean occupancy of a full brick with room for fluctuations
        int ncb_full = R.bd[0] * R.bd[1] * R.bd[2];
        double per_cell = (double)d.n / (double)ncell;
        double own_mean = per_cell * ncb_full;
        R.bcap = std::min((int64_t)round_up((int)std::ceil(own_mean * 1.4 + 64.0), 64),
                          std::max<int64_t>(64, d.n));
        if ((int64_t)R.bcap * R.nbrick < d.n) R.bcap = (int32_t)((d.n + R.nbrick - 1) / R.nbrick);
        R.p_off = p_off;
        R.o_off = o_off;
        R.n = d.n;
        R.c_off = c_off;
        R.b_off = b_off;
        p_off += (int64_t)R.nbrick * R.bcap;
        o_off += d.n;
        c_off += R.ncell;
        b_off += R.nbrick;
        nh_max = std::max(nh_max, (R.bd[0] + 2) * (R.bd[1] + 2) * (R.bd[2] + 2));
        ncb_max = std::max(ncb_max, ncb_full);
        bcap_max = std::max(bcap_max, (int)R.bcap);
        ntypes_max = std::max(ntypes_max, (int)d.ntypes);
        double vol = d.L[0] * d.L[1] * d.L[2];
        rho_cell_max = std::max(rho_cell_max, per_cell);
        own_mean_max = std::max(own_mean_max, own_mean);
        k_mean_max = std::max(k_mean_max, (double)d.n / vol * 4.18879020478639 * rl * rl * rl);
        // static tables: brick-major ranks (x fastest inside a brick and across bricks)
        size_t base = Lo.cell_rank.size();
        Lo.cell_rank.resize(base + R.ncell);
        int32_t rank = 0;
        for (int bz = 0; bz < R.nb[2]; ++bz)
            for (int by = 0; by < R.nb[1]; ++by)
                for (int bx = 0; bx < R.nb[0]; ++bx) {
                    Lo.brick_rank0.push_back(rank);
                    int c0[3] = {bx * R.bd[0], by * R.bd[1], bz * R.bd[2]};
                    int e[3];
                    for (int a = 0; a < 3; ++a) e[a] = std::min(R.bd[a], R.nc[a] - c0[a]);
                    for (int lz = 0; lz < e[2]; ++lz)
                        for (int ly = 0; ly < e[1]; ++ly)
                            for (int lx = 0; lx < e[0]; ++lx) {
                                int gx = c0[0] + lx, gy = c0[1] + ly, gz = c0[2] + lz;
                                Lo.cell_rank[base + gx + R.nc[0] * (gy + R.nc[1] * gz)] = rank++;
                            }
                }
        Lo.reps[r] = R;
    }
    if (p_off >= ((int64_t)1 << 31) - 1) return fail(VBC_ERR_ARG, "more than 2^31 slots in total");
    P.ntot = o_off;
    P.nslots = p_off;
    P.ncell_tot = c_off;
    P.nbrick_tot = b_off;
    P.nh_max = nh_max;
    P.ncb_max = ncb_max;
    P.bcap_max = bcap_max;
    P.ntypes_max = ntypes_max;
    P.any_chains = any_chains;
    P.block = opt.block ? opt.block
                        : std::max(128, std::min(512, round_up((int)std::ceil(own_mean_max), 64)));
    P.k_max = opt.k_max ? round_up(opt.k_max, CHUNK)
                        : std::min(65528, round_up((int)std::ceil(k_mean_max * 1.6 + 24.0), CHUNK));
    P.nchunk = P.k_max / CHUNK;
    if (opt.stage_cap) {
        P.stage_cap = opt.stage_cap;
    } else {
        double mean = rho_cell_max * nh_max;
        P.stage_cap = std::min(65504, round_up((int)std::ceil(mean * 1.3 + 96.0), 32));
    }
    opt.k_max = P.k_max;
    opt.block = P.block;
    opt.stage_cap = P.stage_cap;
    opt.brick = brick_target;
    Lo.opt = opt;

    // workspace
    size_t off = 0;
    const int64_t S = P.nslots;
    Lo.o_reps = carve(off, sizeof(RepDev) * nrep);
    Lo.o_cell_rank = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_brick_rank0 = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_cstart0 = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_cstart1 = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_ccnt0 = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_ccnt1 = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_bcnt0 = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_bcnt1 = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_bfill = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_x0 = carve(off, sizeof(double) * 3 * S);
    Lo.o_x1 = carve(off, sizeof(double) * 3 * S);
    Lo.o_v = carve(off, sizeof(double) * 3 * S);
    Lo.o_Fst = carve(off, sizeof(double) * 3 * S);
    Lo.o_xref = carve(off, sizeof(double) * 3 * S);
    Lo.o_tag = carve(off, sizeof(int32_t) * S);
    Lo.o_type = carve(off, sizeof(int32_t) * S);
    Lo.o_lcell = carve(off, S);
    Lo.o_xs = carve(off, sizeof(double) * 3 * S);
    Lo.o_vs = carve(off, sizeof(double) * 3 * S);
    Lo.o_tags = carve(off, sizeof(int32_t) * S);
    Lo.o_types = carve(off, sizeof(int32_t) * S);
    Lo.o_lcells = carve(off, S);
    Lo.o_src = carve(off, sizeof(int32_t) * S);
    Lo.o_inv = carve(off, sizeof(int32_t) * P.ntot);
    Lo.o_smap = carve(off, sizeof(int32_t) * (size_t)P.nbrick_tot * P.stage_cap);
    Lo.o_wmap = carve(off, (size_t)P.nbrick_tot * P.stage_cap);
    Lo.o_stotal = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_nl = carve(off, 16 * (size_t)P.nchunk * S);
    Lo.o_nn = carve(off, sizeof(uint16_t) * S);
    Lo.o_nd = carve(off, sizeof(double) * S);
    Lo.o_sA = carve(off, (P.precision == VBC_FP64 ? 16 : 8) * (size_t)S);
    Lo.o_win = carve(off, P.nbrick_tot);
    Lo.o_part = carve(off, sizeof(double) * 8 * (size_t)P.nbrick_tot);
    Lo.o_flags = carve(off, sizeof(uint32_t) * nrep);
    Lo.o_step = carve(off, sizeof(uint64_t) * nrep);
    Lo.o_stats = carve(off, sizeof(unsigned long long) * 4 * nrep);
    Lo.o_bevals = carve(off, sizeof(unsigned long long) * P.nbrick_tot);
    Lo.o_bentries = carve(off, sizeof(uint32_t) * P.nbrick_tot);
    Lo.bytes = off;
    return VBC_OK;
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

}  // namespace

// The first build after vbc_set_state starts from caller-order input.
static vbc_status ensure_layout(vbc_handle h, hipStream_t s)
{
    if (!h->need_full) return VBC_OK;
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_full_build(h->B, h->P, h->cur, s); }),
            "full build");
    VBC_TRY(h, launch_flags(h->B, h->P, VBC_FLAG_REBUILD | FLAG_FULL, false, s), "flags");
    h->need_full = false;
    h->f_valid = false;
    return VBC_OK;
}

#define VBC_LAYOUT(h, s)                          \
    do {                                          \
        vbc_status _st = ensure_layout(h, s);     \
        if (_st != VBC_OK) return _st;            \
    } while (0)

extern "C" {

vbc_status vbc_workspace_size(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt,
                              size_t *bytes)
{
    if (!bytes) return fail(VBC_ERR_ARG, "bytes is NULL");
    Layout Lo;
    vbc_status st = plan(reps, nrep, opt, Lo);
    if (st != VBC_OK) return st;
    *bytes = Lo.bytes;
    return VBC_OK;
}

vbc_status vbc_create(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt,
                      void *d_ws, size_t ws_bytes, hipStream_t s, vbc_handle *out)
{
    if (!out) return fail(VBC_ERR_ARG, "out is NULL");
    *out = nullptr;
    Layout Lo;
    vbc_status st = plan(reps, nrep, opt, Lo);
    if (st != VBC_OK) return st;
    if (!d_ws) return fail(VBC_ERR_ARG, "workspace is NULL");
    if (((uintptr_t)d_ws) & 255) return fail(VBC_ERR_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < Lo.bytes)
        return fail(VBC_ERR_CAPACITY, "workspace too small: need " + std::to_string(Lo.bytes) + " bytes");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    int lds_max = 0;
    e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipDeviceGetAttribute");
    size_t need = std::max(std::max(lds_bytes_nlist(Lo.P), lds_bytes_count(Lo.P)),
                           std::max(std::max(lds_bytes_embed(Lo.P), lds_bytes_force(Lo.P)),
                                    lds_bytes_sort(Lo.P)));
    if (need + 2048 > (size_t)lds_max)
        return fail(VBC_ERR_CAPACITY, "staging needs " + std::to_string(need) +
                                          " bytes of LDS per workgroup; the device allows " +
                                          std::to_string(lds_max) + " (lower brick or stage_cap)");

    vbc_handle h = new (std::nothrow) vbc_handle_s;
    if (!h) return fail(VBC_ERR_ARG, "out of host memory");
    h->P = Lo.P;
    h->reps = Lo.reps;
    h->opt = Lo.opt;
    Buffers &B = h->B;
    B.reps = at<RepDev>(d_ws, Lo.o_reps);
    B.cell_rank = at<int32_t>(d_ws, Lo.o_cell_rank);
    B.brick_rank0 = at<int32_t>(d_ws, Lo.o_brick_rank0);
    B.cstart[0] = at<int32_t>(d_ws, Lo.o_cstart0);
    B.cstart[1] = at<int32_t>(d_ws, Lo.o_cstart1);
    B.ccnt[0] = at<int32_t>(d_ws, Lo.o_ccnt0);
    B.ccnt[1] = at<int32_t>(d_ws, Lo.o_ccnt1);
    B.bcnt[0] = at<int32_t>(d_ws, Lo.o_bcnt0);
    B.bcnt[1] = at<int32_t>(d_ws, Lo.o_bcnt1);
    B.bfill = at<int32_t>(d_ws, Lo.o_bfill);
    B.x[0] = at<double>(d_ws, Lo.o_x0);
    B.x[1] = at<double>(d_ws, Lo.o_x1);
    B.v = at<double>(d_ws, Lo.o_v);
    B.Fst = at<double>(d_ws, Lo.o_Fst);
    B.xref = at<double>(d_ws, Lo.o_xref);
    B.tag = at<int32_t>(d_ws, Lo.o_tag);
    B.type = at<int32_t>(d_ws, Lo.o_type);
    B.lcell = at<uint8_t>(d_ws, Lo.o_lcell);
    B.xs = at<double>(d_ws, Lo.o_xs);
    B.vs = at<double>(d_ws, Lo.o_vs);
    B.tags = at<int32_t>(d_ws, Lo.o_tags);
    B.types = at<int32_t>(d_ws, Lo.o_types);
    B.lcells = at<uint8_t>(d_ws, Lo.o_lcells);
    B.src = at<int32_t>(d_ws, Lo.o_src);
    B.inv = at<int32_t>(d_ws, Lo.o_inv);
    B.smap = at<int32_t>(d_ws, Lo.o_smap);
    B.wmap = at<uint8_t>(d_ws, Lo.o_wmap);
    B.stotal = at<int32_t>(d_ws, Lo.o_stotal);
    B.nl = at<uint4>(d_ws, Lo.o_nl);
    B.nn = at<uint16_t>(d_ws, Lo.o_nn);
    B.nd = at<double>(d_ws, Lo.o_nd);
    B.sA = at<void>(d_ws, Lo.o_sA);
    B.win = at<uint8_t>(d_ws, Lo.o_win);
    B.part = at<double>(d_ws, Lo.o_part);
    B.flags = at<uint32_t>(d_ws, Lo.o_flags);
    B.step = at<uint64_t>(d_ws, Lo.o_step);
    B.stats = at<unsigned long long>(d_ws, Lo.o_stats);
    B.bevals = at<unsigned long long>(d_ws, Lo.o_bevals);
    B.bentries = at<uint32_t>(d_ws, Lo.o_bentries);

    // static tables; everything else starts at zero (no particle in any brick)
    e = hipMemsetAsync(d_ws, 0, Lo.bytes, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.reps, Lo.reps.data(), sizeof(RepDev) * nrep, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.cell_rank, Lo.cell_rank.data(), sizeof(int32_t) * Lo.cell_rank.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.brick_rank0, Lo.brick_rank0.data(),
                           sizeof(int32_t) * Lo.brick_rank0.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        vbc_status r = hip_fail(h, e, "vbc_create upload");
        delete h;
        return r;
    }
    *out = h;
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

vbc_status vbc_set_state(vbc_handle h, int32_t rep, const double *d_x, const double *d_v,
                         const int32_t *d_type, uint64_t step0, hipStream_t s)
{
    if (!h || !d_x) return fail(VBC_ERR_ARG, "NULL argument");
    if (rep >= h->P.nrep) {
        h->err = "replica index out of range";
        return VBC_ERR_ARG;
    }
    // a pending full build of other replicas must not see this one half-written
    int64_t n = rep < 0 ? h->P.ntot : h->reps[rep].n;
    int64_t off = rep < 0 ? 0 : h->reps[rep].o_off;
    VBC_TRY(h, launch_set_state(h->B, h->P, h->cur, d_x, d_v, d_type, step0, s, n, off), "set_state");
    h->f_valid = false;
    h->have_state = true;
    h->need_full = true;
    return VBC_OK;
}

vbc_status vbc_get_state(vbc_handle h, int32_t rep, double *d_x, double *d_v, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (rep >= h->P.nrep) {
        h->err = "replica index out of range";
        return VBC_ERR_ARG;
    }
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_LAYOUT(h, s);
    int lo = rep < 0 ? 0 : rep, hi = rep < 0 ? h->P.nrep - 1 : rep;
    int64_t slot_lo = h->reps[lo].p_off;
    int64_t slot_hi = h->reps[hi].p_off + (int64_t)h->reps[hi].nbrick * h->reps[hi].bcap;
    int64_t out_off = h->reps[lo].o_off;
    int64_t out_stride = rep < 0 ? h->P.ntot : h->reps[rep].n;
    VBC_TRY(h, launch_get_state(h->B, h->P, h->cur, slot_lo, slot_hi - slot_lo, out_off, out_stride,
                                d_x, d_v, s),
            "get_state");
    return VBC_OK;
}

vbc_status vbc_build_nlist(vbc_handle h, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    if (h->need_full) {
        VBC_LAYOUT(h, s);
        return VBC_OK;
    }
    VBC_TRY(h, launch_flags(h->B, h->P, VBC_FLAG_REBUILD, true, s), "flags");
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, launch_flags(h->B, h->P, VBC_FLAG_REBUILD, false, s), "flags");
    h->f_valid = false;
    return VBC_OK;
}

vbc_status vbc_count(vbc_handle h, double *d_n, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_LAYOUT(h, s);
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, h->cur, d_n, 0, s); }), "count");
    return VBC_OK;
}

static StepArgs no_step()
{
    StepArgs st;
    std::memset(&st, 0, sizeof(st));
    return st;
}

// count, embed and force of the current positions into Fst (and the optional outputs)
static vbc_status eval_forces(vbc_handle h, bool thermo, const StepArgs &st, double *d_F, double *d_e,
                              hipStream_t s)
{
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, h->cur, nullptr, 0, s); }), "count");
    VBC_TRY(h, timed(h, VBC_K_EMBED, s, [&] { return launch_embed(h->B, h->P, h->cur, s); }), "embed");
    VBC_TRY(h, timed(h, VBC_K_FORCE, s, [&] {
                return launch_force(h->B, h->P, h->cur, MODE_EVAL, thermo, st, d_F, d_e, s);
            }),
            "force");
    return VBC_OK;
}

vbc_status vbc_force(vbc_handle h, double *d_F, double *d_e, double *d_UW, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_LAYOUT(h, s);
    bool thermo = d_e || d_UW;
    vbc_status st = eval_forces(h, thermo, no_step(), d_F, d_e, s);
    if (st != VBC_OK) return st;
    if (d_UW)
        VBC_TRY(h, timed(h, VBC_K_REDUCE, s, [&] { return launch_reduce(h->B, h->P, d_UW, s); }),
                "reduce");
    h->f_valid = true;
    return VBC_OK;
}

// One mid-call step (list rebuild when due, count, dU/dn, force with the closing kick of
// this step and the opening of the next) from position buffer c, on stream s.
static hipError_t launch_mid_step(vbc_handle h, int c, const StepArgs &st, hipStream_t s)
{
    hipError_t e = launch_rebuild(h->B, h->P, c, s);
    if (e == hipSuccess) e = launch_count(h->B, h->P, c, nullptr, 1, s);
    if (e == hipSuccess) e = launch_embed(h->B, h->P, c, s);
    if (e == hipSuccess) e = launch_force(h->B, h->P, c, MODE_MID, false, st, nullptr, nullptr, s);
    return e;
}

static bool same_step_args(const StepArgs &a, const StepArgs &b)
{
    return a.kind == b.kind && a.dt == b.dt && a.hdt == b.hdt && a.c1 == b.c1 && a.c2s == b.c2s &&
           a.seed == b.seed;
}

// Graph of GRAPH_STEPS mid-call steps starting from buffer c, captured once per integrator
// setting on a private stream and launched on the caller's stream.  It holds kernel nodes
// only; every data-dependent choice (rebuild or not) is taken on the GPU.
static hipError_t step_graph(vbc_handle h, int c, const StepArgs &st, hipGraphExec_t *out)
{
    if (h->gexec[c] && same_step_args(h->gst[c], st)) {
        *out = h->gexec[c];
        return hipSuccess;
    }
    if (h->gexec[c]) {
        (void)hipGraphExecDestroy(h->gexec[c]);
        h->gexec[c] = nullptr;
    }
    hipError_t e = hipSuccess;
    if (!h->cap_stream) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int cc = c;
    hipError_t le = hipSuccess;
    for (int k = 0; k < GRAPH_STEPS && le == hipSuccess; ++k) {
        le = launch_mid_step(h, cc, st, h->cap_stream);
        cc ^= 1;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap_stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec[c], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->gexec[c] = nullptr;
        return e;
    }
    h->gst[c] = st;
    *out = h->gexec[c];
    return hipSuccess;
}

vbc_status vbc_step(vbc_handle h, int32_t nsteps, const vbc_integrator *it, hipStream_t s)
{
    if (!h || !it) return fail(VBC_ERR_ARG, "NULL argument");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    if (nsteps < 0) { h->err = "nsteps must be >= 0"; return VBC_ERR_ARG; }
    if (it->kind != VBC_NVE && it->kind != VBC_LANGEVIN) { h->err = "bad integrator kind"; return VBC_ERR_ARG; }
    if (!(it->dt > 0.0) || !std::isfinite(it->dt)) { h->err = "dt must be > 0"; return VBC_ERR_ARG; }
    if (it->kind == VBC_LANGEVIN && (!(it->gamma >= 0.0) || !(it->kT >= 0.0))) {
        h->err = "gamma and kT must be >= 0";
        return VBC_ERR_ARG;
    }
    if (nsteps == 0) return VBC_OK;
    VBC_LAYOUT(h, s);
    StepArgs st = no_step();
    st.kind = it->kind;
    st.dt = it->dt;
    st.hdt = 0.5 * it->dt;
    // same expressions as the plain integrator: c1 = exp(-gamma dt), c2s = sqrt(1-c1^2) sqrt(kT)
    st.c1 = std::exp(-it->gamma * it->dt);
    st.c2s = std::sqrt(1.0 - st.c1 * st.c1) * std::sqrt(it->kT);
    st.seed = it->seed;
    if (!h->f_valid) {
        vbc_status r = eval_forces(h, false, st, nullptr, nullptr, s);
        if (r != VBC_OK) return r;
    }
    // opening half-kick and drift of the first step, from the stored forces
    VBC_TRY(h, timed(h, VBC_K_KICK, s, [&] { return launch_kick_drift(h->B, h->P, h->cur, st, s); }), "kick");
    h->cur ^= 1;
    // nsteps - 1 mid-call steps: whole graphs, then single steps; kernel timing needs the
    // individual launches, so it bypasses the graphs
    int mid = nsteps - 1;
    if (h->use_graphs && !h->prof && mid >= GRAPH_STEPS) {
        hipGraphExec_t ge = nullptr;
        VBC_TRY(h, step_graph(h, h->cur, st, &ge), "step graph");
        for (; mid >= GRAPH_STEPS; mid -= GRAPH_STEPS) VBC_TRY(h, hipGraphLaunch(ge, s), "graph launch");
    }
    for (; mid > 0; --mid) {
        VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
        VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, h->cur, nullptr, 1, s); }), "count");
        VBC_TRY(h, timed(h, VBC_K_EMBED, s, [&] { return launch_embed(h->B, h->P, h->cur, s); }), "embed");
        VBC_TRY(h, timed(h, VBC_K_FORCE, s, [&] {
                    return launch_force(h->B, h->P, h->cur, MODE_MID, false, st, nullptr, nullptr, s);
                }),
                "force");
        h->cur ^= 1;
    }
    // last step: closing half-kick only; its forces are kept for the next call
    VBC_TRY(h, timed(h, VBC_K_BUILD, s, [&] { return launch_rebuild(h->B, h->P, h->cur, s); }), "rebuild");
    VBC_TRY(h, timed(h, VBC_K_COUNT, s, [&] { return launch_count(h->B, h->P, h->cur, nullptr, 1, s); }), "count");
    VBC_TRY(h, timed(h, VBC_K_EMBED, s, [&] { return launch_embed(h->B, h->P, h->cur, s); }), "embed");
    VBC_TRY(h, timed(h, VBC_K_FORCE, s, [&] {
                return launch_force(h->B, h->P, h->cur, MODE_LAST, false, st, nullptr, nullptr, s);
            }),
            "force");
    h->f_valid = true;
    return VBC_OK;
}

vbc_status vbc_check(vbc_handle h, hipStream_t s, uint32_t *flags_per_replica)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    std::vector<uint32_t> f(h->P.nrep);
    VBC_TRY(h, hipMemcpy(f.data(), h->B.flags, sizeof(uint32_t) * h->P.nrep, hipMemcpyDeviceToHost),
            "flags readback");
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
    VBC_TRY(h, launch_flags(h->B, h->P, errs, false, s), "flags");
    VBC_TRY(h, hipStreamSynchronize(s), "sync");
    return st;
}

vbc_status vbc_get_nlist(vbc_handle h, int32_t rep, int32_t *d_pairs, int64_t cap, int64_t *d_count,
                         hipStream_t s)
{
    if (!h || !d_count || (cap > 0 && !d_pairs)) return fail(VBC_ERR_ARG, "NULL argument");
    if (rep < 0 || rep >= h->P.nrep) { h->err = "replica index out of range"; return VBC_ERR_ARG; }
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_LAYOUT(h, s);
    VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
    VBC_TRY(h, launch_export_nlist(h->B, h->P, rep, h->reps[rep].nbrick, d_pairs, cap, d_count, s),
            "export");
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
        for (int b = 0; b < R.nbrick; ++b) {
            pe += ev[R.b_off + b];
            le += en[R.b_off + b];
        }
        out[r].builds = v[4 * r];
        out[r].list_entries = le;
        out[r].pair_evals = pe;
        out[r].evals = v[4 * r + 3];
    }
    return VBC_OK;
}

vbc_status vbc_profile(vbc_handle h, int32_t enable, int32_t max_launches)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (enable && max_launches <= 0) { h->err = "max_launches must be > 0"; return VBC_ERR_ARG; }
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

}  // extern "C"
