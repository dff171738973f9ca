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
    int cur = 0;          // which position buffer holds the current positions
    bool f_valid = false; // Fst holds the forces of the current positions
    bool have_state = false;
    std::string err;
};

namespace {

thread_local std::string g_err;

struct Layout {
    Launch P;
    std::vector<RepDev> reps;
    std::vector<int32_t> cell_rank, brick_rank0;
    vbc_options opt;
    size_t bytes = 0;
    // byte offsets into the workspace
    size_t o_reps, o_cell_rank, o_brick_rank0, o_cell_cnt, o_cell_start, o_x0, o_x1, o_v, o_Fst,
        o_xref, o_tag, o_type, o_pcell, o_inv, o_slot, o_perm, o_xs, o_vs, o_tags, o_types,
        o_pcs, o_nl, o_nn, o_nd, o_sA, o_win, o_part, o_flags, o_step;
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
    if (opt.k_max < 0 || opt.k_max > 65535) return fail(VBC_ERR_ARG, "k_max must be 0..65535");
    if (opt.stage_cap < 0 || opt.stage_cap > 65535)
        return fail(VBC_ERR_ARG, "stage_cap must be 0..65535");

    Launch &P = Lo.P;
    std::memset(&P, 0, sizeof(P));
    P.nrep = nrep;
    P.precision = opt.precision;
    int brick_target = opt.brick ? opt.brick : (opt.precision == VBC_FP64 ? 3 : 4);
    double rho_cell_max = 0.0, k_mean_max = 0.0;
    int64_t p_off = 0;
    int32_t c_off = 0, cs_off = 0, b_off = 0;
    int nh_max = 1, ntypes_max = 1, any_chains = 0;
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
        R.p_off = p_off;
        R.o_off = p_off;
        R.n = d.n;
        R.c_off = c_off;
        R.cs_off = cs_off;
        R.b_off = b_off;
        p_off += d.n;
        c_off += R.ncell;
        cs_off += R.ncell + 1;
        b_off += R.nbrick;
        nh_max = std::max(nh_max, (R.bd[0] + 2) * (R.bd[1] + 2) * (R.bd[2] + 2));
        ntypes_max = std::max(ntypes_max, (int)d.ntypes);
        double vol = d.L[0] * d.L[1] * d.L[2];
        rho_cell_max = std::max(rho_cell_max, (double)d.n / (double)ncell);
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
    if (p_off >= ((int64_t)1 << 31)) return fail(VBC_ERR_ARG, "more than 2^31 particles in total");
    P.ntot = p_off;
    P.ncell_tot = c_off;
    P.ncs_tot = cs_off;
    P.nbrick_tot = b_off;
    P.nh_max = nh_max;
    P.ntypes_max = ntypes_max;
    P.any_chains = any_chains;
    P.block = opt.block ? opt.block : 256;
    P.k_max = opt.k_max ? opt.k_max : std::min(65535, ((int)std::ceil(k_mean_max * 1.6 + 24.0) + 7) / 8 * 8);
    if (opt.stage_cap) {
        P.stage_cap = opt.stage_cap;
    } else {
        double mean = rho_cell_max * nh_max;
        int cap = ((int)std::ceil(mean * 1.5 + 64.0) + 63) / 64 * 64;
        P.stage_cap = std::min(65535, cap);
    }
    opt.k_max = P.k_max;
    opt.block = P.block;
    opt.stage_cap = P.stage_cap;
    opt.brick = brick_target;
    Lo.opt = opt;

    // workspace
    size_t off = 0;
    const int64_t n = P.ntot;
    Lo.o_reps = carve(off, sizeof(RepDev) * nrep);
    Lo.o_cell_rank = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_brick_rank0 = carve(off, sizeof(int32_t) * P.nbrick_tot);
    Lo.o_cell_cnt = carve(off, sizeof(int32_t) * P.ncell_tot);
    Lo.o_cell_start = carve(off, sizeof(int64_t) * P.ncs_tot);
    Lo.o_x0 = carve(off, sizeof(double) * 3 * n);
    Lo.o_x1 = carve(off, sizeof(double) * 3 * n);
    Lo.o_v = carve(off, sizeof(double) * 3 * n);
    Lo.o_Fst = carve(off, sizeof(double) * 3 * n);
    Lo.o_xref = carve(off, sizeof(double) * 3 * n);
    Lo.o_tag = carve(off, sizeof(int32_t) * n);
    Lo.o_type = carve(off, sizeof(int32_t) * n);
    Lo.o_pcell = carve(off, sizeof(int32_t) * n);
    Lo.o_inv = carve(off, sizeof(int64_t) * n);
    Lo.o_slot = carve(off, sizeof(int32_t) * n);
    Lo.o_perm = carve(off, sizeof(int32_t) * n);
    Lo.o_xs = carve(off, sizeof(double) * 3 * n);
    Lo.o_vs = carve(off, sizeof(double) * 3 * n);
    Lo.o_tags = carve(off, sizeof(int32_t) * n);
    Lo.o_types = carve(off, sizeof(int32_t) * n);
    Lo.o_pcs = carve(off, sizeof(int32_t) * n);
    Lo.o_nl = carve(off, sizeof(uint16_t) * (size_t)P.k_max * n);
    Lo.o_nn = carve(off, sizeof(uint16_t) * n);
    Lo.o_nd = carve(off, sizeof(double) * n);
    Lo.o_sA = carve(off, (P.precision == VBC_FP64 ? 16 : 8) * (size_t)n);
    Lo.o_win = carve(off, P.nbrick_tot);
    Lo.o_part = carve(off, sizeof(double) * 8 * (size_t)P.nbrick_tot);
    Lo.o_flags = carve(off, sizeof(uint32_t) * nrep);
    Lo.o_step = carve(off, sizeof(uint64_t) * nrep);
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

#define VBC_TRY(h, expr, where)                        \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return hip_fail(h, _e, where); \
    } while (0)

}  // namespace

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
                           std::max(lds_bytes_embed(Lo.P), lds_bytes_force(Lo.P)));
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
    B.cell_cnt = at<int32_t>(d_ws, Lo.o_cell_cnt);
    B.cell_start = at<int64_t>(d_ws, Lo.o_cell_start);
    B.x[0] = at<double>(d_ws, Lo.o_x0);
    B.x[1] = at<double>(d_ws, Lo.o_x1);
    B.v = at<double>(d_ws, Lo.o_v);
    B.Fst = at<double>(d_ws, Lo.o_Fst);
    B.xref = at<double>(d_ws, Lo.o_xref);
    B.tag = at<int32_t>(d_ws, Lo.o_tag);
    B.type = at<int32_t>(d_ws, Lo.o_type);
    B.pcell = at<int32_t>(d_ws, Lo.o_pcell);
    B.inv = at<int64_t>(d_ws, Lo.o_inv);
    B.slot = at<int32_t>(d_ws, Lo.o_slot);
    B.perm = at<int32_t>(d_ws, Lo.o_perm);
    B.xs = at<double>(d_ws, Lo.o_xs);
    B.vs = at<double>(d_ws, Lo.o_vs);
    B.tags = at<int32_t>(d_ws, Lo.o_tags);
    B.types = at<int32_t>(d_ws, Lo.o_types);
    B.pcs = at<int32_t>(d_ws, Lo.o_pcs);
    B.nl = at<uint16_t>(d_ws, Lo.o_nl);
    B.nn = at<uint16_t>(d_ws, Lo.o_nn);
    B.nd = at<double>(d_ws, Lo.o_nd);
    B.sA = at<void>(d_ws, Lo.o_sA);
    B.win = at<uint8_t>(d_ws, Lo.o_win);
    B.part = at<double>(d_ws, Lo.o_part);
    B.flags = at<uint32_t>(d_ws, Lo.o_flags);
    B.step = at<uint64_t>(d_ws, Lo.o_step);

    // static tables; everything else starts at zero
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

static bool rep_range(vbc_handle h, int32_t rep, int &lo, int &hi, int64_t &n, int64_t &off)
{
    if (rep < 0) {
        lo = 0;
        hi = h->P.nrep - 1;
        n = h->P.ntot;
        off = 0;
        return true;
    }
    if (rep >= h->P.nrep) return false;
    lo = hi = rep;
    n = h->reps[rep].n;
    off = h->reps[rep].o_off;
    return true;
}

vbc_status vbc_set_state(vbc_handle h, int32_t rep, const double *d_x, const double *d_v,
                         const int32_t *d_type, uint64_t step0, hipStream_t s)
{
    if (!h || !d_x) return fail(VBC_ERR_ARG, "NULL argument");
    int lo, hi;
    int64_t n, off;
    if (!rep_range(h, rep, lo, hi, n, off)) {
        h->err = "replica index out of range";
        return VBC_ERR_ARG;
    }
    VBC_TRY(h, launch_set_state(h->B, h->P, lo, hi, d_x, d_v, d_type, step0, s, n, off), "set_state");
    // both position buffers were written: either may serve as current
    h->f_valid = false;
    h->have_state = true;
    return VBC_OK;
}

vbc_status vbc_get_state(vbc_handle h, int32_t rep, double *d_x, double *d_v, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    int lo, hi;
    int64_t n, off;
    if (!rep_range(h, rep, lo, hi, n, off)) {
        h->err = "replica index out of range";
        return VBC_ERR_ARG;
    }
    VBC_TRY(h, launch_get_state(h->B, h->P, h->cur, lo, hi, d_x, d_v, s, n, off), "get_state");
    return VBC_OK;
}

vbc_status vbc_build_nlist(vbc_handle h, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_TRY(h, launch_flags(h->B, h->P, VBC_FLAG_REBUILD, true, s), "flags");
    VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
    VBC_TRY(h, launch_flags(h->B, h->P, VBC_FLAG_REBUILD, false, s), "flags");
    h->f_valid = false;
    return VBC_OK;
}

vbc_status vbc_count(vbc_handle h, double *d_n, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
    VBC_TRY(h, launch_count(h->B, h->P, h->cur, d_n, s), "count");
    h->f_valid = false;
    return VBC_OK;
}

static StepArgs no_step()
{
    StepArgs st;
    std::memset(&st, 0, sizeof(st));
    return st;
}

vbc_status vbc_force(vbc_handle h, double *d_F, double *d_e, double *d_UW, hipStream_t s)
{
    if (!h) return fail(VBC_ERR_ARG, "NULL handle");
    if (!h->have_state) { h->err = "no state set"; return VBC_ERR_STATE; }
    bool thermo = d_e || d_UW;
    VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
    VBC_TRY(h, launch_count(h->B, h->P, h->cur, nullptr, s), "count");
    VBC_TRY(h, launch_embed(h->B, h->P, h->cur, s), "embed");
    VBC_TRY(h, launch_force(h->B, h->P, h->cur, MODE_EVAL, thermo, no_step(), d_F, d_e, s), "force");
    if (d_UW) VBC_TRY(h, launch_reduce(h->B, h->P, d_UW, s), "reduce");
    h->f_valid = true;
    return VBC_OK;
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
    StepArgs st = no_step();
    st.kind = it->kind;
    st.dt = it->dt;
    st.hdt = 0.5 * it->dt;
    // same expressions as the plain integrator: c1 = exp(-gamma dt), c2s = sqrt(1-c1^2) sqrt(kT)
    st.c1 = std::exp(-it->gamma * it->dt);
    st.c2s = std::sqrt(1.0 - st.c1 * st.c1) * std::sqrt(it->kT);
    st.seed = it->seed;
    if (!h->f_valid) {
        VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
        VBC_TRY(h, launch_count(h->B, h->P, h->cur, nullptr, s), "count");
        VBC_TRY(h, launch_embed(h->B, h->P, h->cur, s), "embed");
        VBC_TRY(h, launch_force(h->B, h->P, h->cur, MODE_EVAL, false, st, nullptr, nullptr, s), "force");
    }
    st.step_off = 0;
    VBC_TRY(h, launch_kick_drift(h->B, h->P, h->cur, st, s), "kick");
    h->cur ^= 1;
    for (int k = 0; k < nsteps; ++k) {
        VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
        VBC_TRY(h, launch_count(h->B, h->P, h->cur, nullptr, s), "count");
        VBC_TRY(h, launch_embed(h->B, h->P, h->cur, s), "embed");
        bool last = (k == nsteps - 1);
        st.step_off = (uint64_t)k + 1;
        VBC_TRY(h, launch_force(h->B, h->P, h->cur, last ? MODE_LAST : MODE_MID, false, st, nullptr,
                                nullptr, s),
                "force");
        if (!last) h->cur ^= 1;
    }
    VBC_TRY(h, launch_advance(h->B, h->P, (uint64_t)nsteps, s), "advance");
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
    if (flags_per_replica) std::memcpy(flags_per_replica, f.data(), sizeof(uint32_t) * h->P.nrep);
    vbc_status st = VBC_OK;
    for (int r = 0; r < h->P.nrep && st == VBC_OK; ++r) {
        if (f[r] & VBC_FLAG_NONFINITE) {
            st = VBC_ERR_NONFINITE;
            h->err = "replica " + std::to_string(r) + ": non-finite coordinates or forces";
        } else if (f[r] & VBC_FLAG_NLIST_OVERFLOW) {
            st = VBC_ERR_NLIST_OVERFLOW;
            h->err = "replica " + std::to_string(r) + ": neighbour list overflow (raise k_max)";
        } else if (f[r] & VBC_FLAG_STAGE_OVERFLOW) {
            st = VBC_ERR_CAPACITY;
            h->err = "replica " + std::to_string(r) + ": brick staging overflow (raise stage_cap)";
        }
    }
    uint32_t errs = VBC_FLAG_NONFINITE | VBC_FLAG_NLIST_OVERFLOW | VBC_FLAG_STAGE_OVERFLOW;
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
    VBC_TRY(h, launch_rebuild(h->B, h->P, h->cur, s), "rebuild");
    VBC_TRY(h, launch_export_nlist(h->B, h->P, rep, h->reps[rep].nbrick, d_pairs, cap, d_count, s),
            "export");
    return VBC_OK;
}

}  // extern "C"
