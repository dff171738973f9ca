// vbc_kernels.hip -- gfx950 kernels of the VBC hot path.
//
// Passes (Section 2, paragraph on the cost of the correction: a count sweep and a force
// sweep of the neighbour list; the force itself follows from differentiating eq. (Vhat)):
//   count  : n_i = sum_j omega(r_ij, r_l, r_h)                       eq. (counter)
//            s_i = omega(n_i, f - delta, f - delta + 1)              eq. (Psi), (Psidelta)
//   embed  : A_i = dU/dn_i = s'_i sum_j s_j V_a(r_ij), only for particles whose count lies
//            inside the switching window (elsewhere s'_i = 0); a workgroup whose brick holds
//            no such particle exits at once
//   force  : phi_ij = V_r'(r) + s_i s_j V_a'(r) + (A_i + A_j) c'(r),  F_i = -sum_j phi_ij r_hat_ij
//            plus the integrator update of the particle, fused in the same pass.
// The energy gradient needs A of every counted neighbour, which is only final once all
// counts are, hence the separate sparse embed pass between the two list sweeps.
//
// List build (when some particle has moved more than half the buffer): every workgroup
// gathers the particles now inside its brick from the one-cell halo of the previous
// layout, orders them by (cell, tag) in LDS and writes the next layout; a second kernel
// copies each brick to the live arrays and builds its list.  Starting from unsorted input
// (after vbc_set_state), particles are first binned into per-brick buckets with atomics.
//
// Data flow of one workgroup in a pass: it owns one brick; it stages its own particles and
// the halo into LDS in a brick-local frame, then sweeps each own particle's list (16-bit
// indices into the staging order, eight per 16-byte chunk) reading neighbours from LDS.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <tuple>

#include "vbc_internal.h"

namespace vbc {

#define VBC_WAVE 64
#define VBC_GROUP 8  // lanes that copy one cell during staging

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <class T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };
template <class T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

// Pair arithmetic: the hardware square root and reciprocal square root in FP32 (<= 1 ulp),
// the exactly rounded ones in FP64.
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float clamp01(float u) { return __builtin_amdgcn_fmed3f(u, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double u) { return fmin(fmax(u, 0.0), 1.0); }

// Map workgroups to bricks so that consecutive bricks (which share halo cells) land on
// the same XCD: workgroups are dealt round-robin over the 8 XCDs, so workgroup g runs on
// XCD g % 8; give that XCD a contiguous run of the T bricks to visit.  The grid is padded
// to a multiple of 8, at least T.  The bricks are either the contiguous range
// [b_lo, b_lo + nb_launch) (P.list < 0: all bricks, or one replica's) or the entries of
// work list P.list, which the step computes on the GPU.  Returns false for a workgroup
// with nothing to do (padding, or a free brick).
__device__ __forceinline__ bool brick_of_block(const Launch &P, const Buffers &B, int &b)
{
    const int g = blockIdx.x, j = g >> 3;
    const int T = P.list < 0 ? P.nb_launch : B.wl_n[P.list];
    const int chunk = (T + 7) >> 3;
    const int k = (g & 7) * chunk + j;
    if (j >= chunk || k >= T) return false;
    b = P.list < 0 ? P.b_lo + k : B.wl[P.list][k];
    return true;
}

__device__ __forceinline__ bool resolve_brick(const Launch &P, const Buffers &B, int &b, int &r)
{
    if (!brick_of_block(P, B, b)) return false;
    r = B.brick_rep[b];
    return r >= 0;
}

// Smooth step of eq. (omega) and its derivative, in FP64 (used for the switching factor).
__device__ __forceinline__ double omega_d64(double x, double x1, double x2)
{
    if (x <= x1) return 1.0;
    if (x >= x2) return 0.0;
    double u = (x - x1) / (x2 - x1);
    double q = 1.0 - u * u;
    return q * q;
}

__device__ __forceinline__ double omega_dd64(double x, double x1, double x2)
{
    if (x <= x1 || x >= x2) return 0.0;
    double w = x2 - x1;
    double u = (x - x1) / w;
    return -4.0 * u * (1.0 - u * u) / w;
}

template <class Real>
__device__ __forceinline__ Real omega_r(Real x, Real x1, Real x2)
{
    Real u = (x - x1) / (x2 - x1);
    u = u < Real(0) ? Real(0) : (u > Real(1) ? Real(1) : u);
    Real q = Real(1) - u * u;
    return q * q;
}

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11): two 32x32->64-bit
// multiplies by fixed odd constants per round, high halves xor-ed with the other two
// counter words and the round key; the key is bumped by two Weyl constants per round.
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        // one 32x32->64-bit product each (a single multiply instruction for both halves)
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Zero-mean unit-variance uniform variates sqrt(3)(2u - 1) from the first three words,
// u = (word + 1/2) 2^-32; key = the halves of seed, counter = the halves of step, then of
// tag: only exactly rounded operations.
__device__ __forceinline__ void langevin_noise(uint64_t seed, uint64_t tag, uint64_t step,
                                               double xi[3])
{
#pragma clang fp contract(off)
    uint32_t c0 = (uint32_t)step, c1 = (uint32_t)(step >> 32), c2 = (uint32_t)tag,
             c3 = (uint32_t)(tag >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double SQRT3 = 1.7320508075688772;
    xi[0] = (2.0 * (((double)c0 + 0.5) * 0x1.0p-32) - 1.0) * SQRT3;
    xi[1] = (2.0 * (((double)c1 + 0.5) * 0x1.0p-32) - 1.0) * SQRT3;
    xi[2] = (2.0 * (((double)c2 + 0.5) * 0x1.0p-32) - 1.0) * SQRT3;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = VBC_WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, VBC_WAVE);
    return v;
}

// Eight sums over the wave at once.  At each of the first three halvings a lane keeps half
// of its values and trades the other half with the lane 32, 16 or 8 away, so that from
// then on every lane carries one value, which three more exchanges finish: ten shuffles
// instead of the 48 of eight separate sums.  Returns, in lane L, the total of value
// 4 b5 + 2 b4 + b3 (the bits of L): value k's total is in lane 8k.  The order of the
// additions is fixed.
__device__ __forceinline__ double wave_sum8(const double (&a)[8])
{
    const int lane = threadIdx.x % VBC_WAVE;
    double s[4], t[2];
    bool hi = lane & 32;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double keep = hi ? a[k + 4] : a[k], give = hi ? a[k] : a[k + 4];
        s[k] = keep + __shfl_xor(give, 32, VBC_WAVE);
    }
    hi = lane & 16;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double keep = hi ? s[k + 2] : s[k], give = hi ? s[k] : s[k + 2];
        t[k] = keep + __shfl_xor(give, 16, VBC_WAVE);
    }
    hi = lane & 8;
    double u = (hi ? t[1] : t[0]) + __shfl_xor(hi ? t[0] : t[1], 8, VBC_WAVE);
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) u += __shfl_xor(u, o, VBC_WAVE);
    return u;
}

// Exclusive scan of a[0..n) in place by the first wave; returns the total (valid in the
// first wave).  Call from all threads of the block between barriers.
__device__ __forceinline__ int wave0_exclusive_scan(int *a, int n)
{
    int carry = 0;
    if (threadIdx.x < VBC_WAVE) {
        int lane = threadIdx.x;
        for (int base = 0; base < n; base += VBC_WAVE) {
            int q = base + lane;
            int v = q < n ? a[q] : 0;
            int incl = v;
#pragma unroll
            for (int o = 1; o < VBC_WAVE; o <<= 1) {
                int t = __shfl_up(incl, o, VBC_WAVE);
                if (lane >= o) incl += t;
            }
            if (q < n) a[q] = carry + incl - v;
            carry += __shfl(incl, VBC_WAVE - 1, VBC_WAVE);
        }
    }
    return carry;
}

// Wrap one coordinate into [0, L).
__device__ __forceinline__ double wrap1(double t, double L)
{
    if (t < 0.0 || t >= L) {
        t = t - L * floor(t / L);
        if (t >= L) t -= L;
        if (t < 0.0) t = 0.0;
    }
    return t;
}

__device__ __forceinline__ int cell_of(double t, double h, int nc)
{
    int c = (int)floor(t / h);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// ---------------------------------------------------------------------------
// brick geometry and staging
// ---------------------------------------------------------------------------

struct StageHdr {
    int64_t base;   // first slot of the brick
    int n_own;
    int total;
    int rank0;
    int nh, ncb;
    int c0[3], e[3], H[3];
    double O[3];
    int overflow;
};

struct StageTabs {
    int *q_off;    // staged offset of each halo-grid cell (own and halo)
    int *q_cnt;    // particles in the cell
    int *q_src;    // first slot of the cell
    int *q_hpre;   // exclusive prefix of halo-cell counts (own cells contribute 0)
    int *q_w;      // packed image shift (wx+1) | (wy+1) << 2 | (wz+1) << 4
};

__device__ __forceinline__ int unpack_w(int w, int a) { return ((w >> (2 * a)) & 3) - 1; }

__device__ __forceinline__ size_t align32(size_t b) { return (b + 31) & ~(size_t)31; }

__device__ __forceinline__ StageTabs carve_tabs(unsigned char *smem, int nh_cap)
{
    StageTabs T;
    int *p = (int *)smem;
    T.q_off = p;
    T.q_cnt = p + nh_cap;
    T.q_src = p + 2 * nh_cap;
    T.q_hpre = p + 3 * nh_cap;
    T.q_w = p + 4 * nh_cap;
    return T;
}

__device__ __forceinline__ unsigned char *after_tabs(unsigned char *smem, int nh_cap)
{
    return smem + align32((size_t)5 * nh_cap * sizeof(int));
}

// Geometry of brick lb of replica R (one thread).
__device__ __forceinline__ void brick_geometry(const RepDev &R, int lb, StageHdr &S)
{
    int Bc[3] = {lb % R.nb[0], (lb / R.nb[0]) % R.nb[1], lb / (R.nb[0] * R.nb[1])};
    S.ncb = 1;
    for (int a = 0; a < 3; ++a) {
        S.c0[a] = Bc[a] * R.bd[a];
        S.e[a] = min(R.bd[a], R.nc[a] - S.c0[a]);
        S.H[a] = S.e[a] + 2;
        S.ncb *= S.e[a];
        S.O[a] = ((double)S.c0[a] + 0.5 * (double)S.e[a]) * R.h[a];
    }
    S.nh = S.H[0] * S.H[1] * S.H[2];
    S.base = R.p_off + (int64_t)lb * R.bcap;
}

// Lay out the staging of brick b (local index lb) of replica R from a set of cell tables:
// own particles first (the brick's slot range), then every halo cell of the (e+2)^3 grid
// in x-fastest order.  All threads of the block call this.
__device__ void stage_tables(const RepDev &R, int b, int lb, const int32_t *brick_rank0,
                             const int32_t *cell_rank, const int32_t *cstart,
                             const int32_t *ccnt, const int32_t *bcnt, StageHdr &S,
                             StageTabs T, int stage_cap)
{
    if (threadIdx.x == 0) {
        brick_geometry(R, lb, S);
        S.rank0 = brick_rank0[b];
        S.n_own = bcnt[b];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.nh; q += blockDim.x) {
        int h[3] = {q % S.H[0], (q / S.H[0]) % S.H[1], q / (S.H[0] * S.H[1])};
        int g[3], w = 0;
        bool own = true;
        for (int a = 0; a < 3; ++a) {
            int ga = S.c0[a] - 1 + h[a];
            int wa = ga < 0 ? -1 : (ga >= R.nc[a] ? 1 : 0);
            g[a] = ga - wa * R.nc[a];
            w |= (wa + 1) << (2 * a);
            own = own && (h[a] >= 1 && h[a] <= S.e[a]);
        }
        int rank = cell_rank[R.c_off + g[0] + R.nc[0] * (g[1] + R.nc[1] * g[2])];
        int st = cstart[R.c_off + rank];
        int cnt = ccnt[R.c_off + rank];
        T.q_src[q] = st;
        T.q_cnt[q] = cnt;
        T.q_w[q] = w;
        T.q_off[q] = own ? (int)(st - S.base) : -1;
        T.q_hpre[q] = own ? 0 : cnt;
    }
    __syncthreads();
    int tot = wave0_exclusive_scan(T.q_hpre, S.nh);
    if (threadIdx.x == 0) {
        S.total = S.n_own + tot;
        S.overflow = S.total > stage_cap;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.nh; q += blockDim.x)
        if (T.q_off[q] < 0) T.q_off[q] = S.n_own + T.q_hpre[q];
    __syncthreads();
}

// Call fn(staged_slot, source_slot, packed_shift) for every staged particle.  Groups of
// eight lanes take one cell at a time, so no search is needed and the loads of all cells
// are in flight together.
template <class F>
__device__ __forceinline__ void stage_copy(const StageHdr &S, const StageTabs &T, F &&fn)
{
    int gid = threadIdx.x / VBC_GROUP, gl = threadIdx.x % VBC_GROUP;
    int ng = blockDim.x / VBC_GROUP;
    for (int q = gid; q < S.nh; q += ng) {
        int off = T.q_off[q], src = T.q_src[q], cnt = T.q_cnt[q], w = T.q_w[q];
        for (int k = gl; k < cnt; k += VBC_GROUP) fn(off + k, src + k, w);
    }
}

// Header of brick b for a pass over the current layout: geometry, own range and the
// staged count recorded by the last list build (one thread).
__device__ __forceinline__ void pass_header(const RepDev &R, const Buffers &B, int b, int lb,
                                            int stage_cap, StageHdr &S)
{
    brick_geometry(R, lb, S);
    S.n_own = B.bcnt[0][b];
    S.total = B.stotal[b];
    S.overflow = S.total > stage_cap;
}

// Call fn(staged_slot, source_slot, packed_shift) for every particle staged by brick b,
// from the staging map the list build recorded: one coalesced read, no cell-table walk.
template <class F>
__device__ __forceinline__ void stage_map(const Buffers &B, int b, int stage_cap,
                                          const StageHdr &S, F &&fn)
{
    const int32_t *sm = B.smap + (size_t)b * stage_cap;
    const uint8_t *wm = B.wmap + (size_t)b * stage_cap;
    for (int t = threadIdx.x; t < S.total; t += blockDim.x) fn(t, sm[t], (int)wm[t]);
}

// stage_map with four staged particles per thread at a time: the map reads of all four go
// out first, then fn(staged_slot, source_slot, packed_shift, valid) for each; fn must do
// its own loads unconditionally (the indices are clamped into the staging) and guard only
// its stores with valid, so that the gathers of the four overlap.
//
// The map entries of the first four (threadIdx.x + j blockDim.x) are read by map_prefetch
// as soon as the brick is known, before its header: their latency then overlaps the
// header's, and the gathers can go out as soon as the header is known.  Entries past the
// staged count are stale but valid slot indices (the map is cleared at creation and only
// ever holds slots), and their stores are not made.
struct MapFirst {
    int src[4], w[4];
};

__device__ __forceinline__ MapFirst map_prefetch(const Buffers &B, int b, int stage_cap)
{
    const int32_t *sm = B.smap + (size_t)b * stage_cap;
    const uint8_t *wm = B.wmap + (size_t)b * stage_cap;
    MapFirst m;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = min((int)(threadIdx.x + j * blockDim.x), stage_cap - 1);
        m.src[j] = sm[t];
        m.w[j] = (int)wm[t];
    }
    return m;
}

template <class F>
__device__ __forceinline__ void stage_map4(const Buffers &B, int b, int stage_cap, const StageHdr &S,
                                           const MapFirst &first, F &&fn)
{
    const int32_t *sm = B.smap + (size_t)b * stage_cap;
    const uint8_t *wm = B.wmap + (size_t)b * stage_cap;
    const int nt = blockDim.x, last = S.total - 1;
    for (int t0 = threadIdx.x; t0 < S.total; t0 += 4 * nt) {
        int src[4], w[4];
        if (t0 == (int)threadIdx.x) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                src[j] = first.src[j];
                w[j] = first.w[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = min(t0 + j * nt, last);
                src[j] = sm[t];
                w[j] = (int)wm[t];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) fn(t0 + j * nt, src[j], w[j], t0 + j * nt < S.total);
    }
}

// ---------------------------------------------------------------------------
// state in / out, flags
// ---------------------------------------------------------------------------

// Caller-order input of replica r (element tag at in_off + tag of each stride-in_stride
// component array) into the live arrays at slot p_off + tag: the unsorted layout that the
// next full build starts from.
__global__ void k_set_state(Buffers B, int64_t S_, int cur, int r, int64_t in_off,
                            int64_t in_stride, const double *__restrict__ x,
                            const double *__restrict__ v, const int32_t *__restrict__ type,
                            uint64_t step0)
{
    const RepDev &R = B.reps[r];
    int64_t tg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tg >= R.n) return;
    int64_t i = in_off + tg;
    int64_t d = R.p_off + tg;
    for (int a = 0; a < 3; ++a) {
        B.x[cur][3 * d + a] = x[a * in_stride + i];
        B.v[a * S_ + d] = v ? v[a * in_stride + i] : 0.0;
    }
    B.tag[d] = (int32_t)tg;
    int ty = type ? type[i] : 0;
    B.type[d] = (ty >= 0 && ty < R.ntypes) ? ty : 0;
    if (tg == 0) {
        B.step[r] = step0;
        B.flags[r] = VBC_FLAG_REBUILD | FLAG_FULL;
    }
}

// Live state of replica r out in caller order (element out_off + tag).
__global__ void k_get_state(Buffers B, int64_t S_, int cur, int r, int64_t out_off,
                            int64_t out_stride, double *__restrict__ x, double *__restrict__ v)
{
    const RepDev &R = B.reps[r];
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)R.nbrick * R.bcap) return;
    int lb = (int)(k / R.bcap);
    if (k - (int64_t)lb * R.bcap >= B.bcnt[0][R.b_off + lb]) return;
    int64_t slot = R.p_off + k;
    int64_t dst = out_off + B.tag[slot];
    for (int a = 0; a < 3; ++a) {
        if (x) x[a * out_stride + dst] = wrap1(B.x[cur][3 * slot + a], R.L[a]);
        if (v) v[a * out_stride + dst] = B.v[a * S_ + slot];
    }
}

__global__ void k_flags(Buffers B, int r_lo, int r_n, uint32_t bits, int set)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= r_n) return;
    r += r_lo;
    if (set) B.flags[r] |= bits; else B.flags[r] &= ~bits;
}

// Rank of a cell in the brick-major order (bricks x-fastest, cells x-fastest inside a
// brick; edge bricks are cut by the box): every brick before brick (bx, by, bz) covers,
// whole, the z-slabs below its first cell, the rows below it in its own slab and the
// columns before it in its own row.
__device__ __forceinline__ int32_t brick_major_rank(const RepDev &R, const int g[3])
{
    int c0[3], e[3], l[3];
    for (int a = 0; a < 3; ++a) {
        c0[a] = g[a] / R.bd[a] * R.bd[a];
        e[a] = min(R.bd[a], R.nc[a] - c0[a]);
        l[a] = g[a] - c0[a];
    }
    int64_t rank0 = (int64_t)c0[2] * R.nc[0] * R.nc[1] + (int64_t)c0[1] * R.nc[0] * e[2] +
                    (int64_t)c0[0] * e[1] * e[2];
    return (int32_t)(rank0 + l[0] + e[0] * (l[1] + e[1] * l[2]));
}

// A replica enters the workspace: its static tables (brick owner, brick-major cell ranks)
// and cleared per-brick, per-cell and per-replica state.
__global__ void k_admit(Buffers B, int r)
{
    const RepDev &R = B.reps[r];
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < R.nbrick) {
        int lb = (int)t, b = R.b_off + lb;
        int g[3] = {lb % R.nb[0] * R.bd[0], lb / R.nb[0] % R.nb[1] * R.bd[1],
                    lb / (R.nb[0] * R.nb[1]) * R.bd[2]};
        B.brick_rep[b] = r;
        B.brick_rank0[b] = brick_major_rank(R, g);
        B.bcnt[0][b] = 0;
        B.bcnt[1][b] = 0;
        B.bfill[b] = 0;
        B.stotal[b] = 0;
        B.wcnt[b] = 0;
        for (int k = 0; k < 8; ++k) B.part[(size_t)b * 8 + k] = 0.0;
        B.bevals[b] = 0ull;
        B.bentries[b] = 0u;
    }
    if (t < R.ncell) {
        int c = (int)t;
        int g[3] = {c % R.nc[0], c / R.nc[0] % R.nc[1], c / (R.nc[0] * R.nc[1])};
        int64_t k = R.c_off + c;
        B.cell_rank[k] = brick_major_rank(R, g);
        B.cstart[0][k] = 0;
        B.cstart[1][k] = 0;
        B.ccnt[0][k] = 0;
        B.ccnt[1][k] = 0;
    }
    if (t == 0) {
        B.flags[r] = 0u;
        B.step[r] = 0ull;
        for (int k = 0; k < 4; ++k) B.stats[4 * r + k] = 0ull;
    }
}

// A replica leaves: its bricks become free (brick kernels skip them) and its descriptor
// empty (reductions over it give zeros).
__global__ void k_retire(Buffers B, int r, int b_off, int nbrick)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nbrick) B.brick_rep[b_off + t] = -1;
    if (t == 0) {
        B.reps[r].n = 0;
        B.reps[r].nbrick = 0;
        B.reps[r].ncell = 0;
    }
}

// Device time stamp at the end of a step (stream order: after every kernel of the step).
__global__ void k_stamp(Buffers B, uint32_t mask)
{
    unsigned long long k = B.stamp_n[0];
    B.stamps[k & mask] = wall_clock64();
    B.stamp_n[0] = k + 1ull;
}

// Work lists of the capacity-wide launches, made on the GPU at the start of every step
// from the replica table: list 0 = every brick of every live replica, list 1 = the bricks
// of the replicas whose list is due for an incremental rebuild.  Replica slots in order,
// bricks in order inside a replica, so consecutive entries are neighbouring bricks.
__global__ void __launch_bounds__(1024) k_worklist(Buffers B, int nrep)
{
    __shared__ int pre[2][MAX_REPLICAS + 1];
    __shared__ int boff[MAX_REPLICAS];
    __shared__ int tot[2];
    for (int r = threadIdx.x; r < nrep; r += blockDim.x) {
        const RepDev &R = B.reps[r];
        const int nb = R.nbrick;  // 0 for a free slot
        const uint32_t fl = B.flags[r];
        pre[0][r] = nb;
        pre[1][r] = ((fl & VBC_FLAG_REBUILD) && !(fl & FLAG_FULL)) ? nb : 0;
        boff[r] = R.b_off;
    }
    __syncthreads();
    const int t0 = wave0_exclusive_scan(pre[0], nrep);
    const int t1 = wave0_exclusive_scan(pre[1], nrep);
    if (threadIdx.x == 0) {
        tot[0] = t0;
        tot[1] = t1;
        B.wl_n[0] = t0;
        B.wl_n[1] = t1;
    }
    __syncthreads();
    for (int l = 0; l < 2; ++l) {
        const int T = tot[l];
        for (int k = threadIdx.x; k < T; k += blockDim.x) {
            // the last replica whose first entry is <= k (empty entries share their
            // successor's start, so the one found has bricks)
            int lo = 0, hi = nrep - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (pre[l][mid] <= k) lo = mid; else hi = mid - 1;
            }
            B.wl[l][k] = boff[lo] + (k - pre[l][lo]);
        }
    }
}

// ---------------------------------------------------------------------------
// list build, step 1: the next sorted layout
// ---------------------------------------------------------------------------

struct SortTabs {
    int *m_src;    // [bcap] source slot of each member
    int *m_tag;    // [bcap]
    int *m_lc;     // [bcap] cell inside the brick
    int *bucket;   // [bcap] members grouped by cell
    int *hist;     // [ncb_max]
    int *cpre;     // [ncb_max]
    int *fill;     // [ncb_max]
};

__device__ __forceinline__ SortTabs carve_sort(unsigned char *p, int bcap, int ncb_max)
{
    SortTabs T;
    int *q = (int *)p;
    T.m_src = q;
    T.m_tag = q + bcap;
    T.m_lc = q + 2 * bcap;
    T.bucket = q + 3 * bcap;
    T.hist = q + 4 * bcap;
    T.cpre = T.hist + ncb_max;
    T.fill = T.cpre + ncb_max;
    return T;
}

// Order the nmem members gathered in LDS by (cell, tag), then write them in that order
// into the next layout of brick b, with the brick's cell tables.  Positions are wrapped
// into the box as they are copied.  On entry hist holds the members per cell, cpre a
// copy of it and fill zeros.
__device__ void place_members(const Buffers &B, const RepDev &R, int r, int b,
                              const StageHdr &S, SortTabs T, int nmem, int cur, int64_t S_)
{
    wave0_exclusive_scan(T.cpre, S.ncb);
    __syncthreads();
    for (int m = threadIdx.x; m < nmem; m += blockDim.x) {
        int lc = T.m_lc[m];
        int p = T.cpre[lc] + atomicAdd(&T.fill[lc], 1);
        T.bucket[p] = m;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < nmem; p += blockDim.x) {
        int m = T.bucket[p];
        int lc = T.m_lc[m];
        int lo = T.cpre[lc], hi = lo + T.hist[lc];
        int key = T.m_tag[m];
        int rank = 0;
        for (int k = lo; k < hi; ++k) rank += (T.m_tag[T.bucket[k]] < key) ? 1 : 0;
        int64_t ns = S.base + lo + rank;
        int64_t o = T.m_src[m];
        for (int a = 0; a < 3; ++a) {
            B.xs[3 * ns + a] = wrap1(B.x[cur][3 * o + a], R.L[a]);
            B.vs[a * S_ + ns] = B.v[a * S_ + o];
        }
        B.tags[ns] = key;
        B.types[ns] = B.type[o];
        B.lcells[ns] = (uint8_t)lc;
        // caller index -> slot: read only for the bond partners of chains (a scattered
        // write per particle, left out without bonds)
        if (R.chain_len > 1) B.inv[R.o_off + key] = (int32_t)ns;
    }
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) {
        B.cstart[1][R.c_off + S.rank0 + lc] = (int32_t)(S.base + T.cpre[lc]);
        B.ccnt[1][R.c_off + S.rank0 + lc] = T.hist[lc];
    }
    if (threadIdx.x == 0) B.bcnt[1][b] = nmem;
}

// Local cell of position x inside brick S, or -1 if the particle is not in the brick.
__device__ __forceinline__ int local_cell(const RepDev &R, const StageHdr &S, const double *xw)
{
    int l[3];
    for (int a = 0; a < 3; ++a) {
        int c = cell_of(xw[a], R.h[a], R.nc[a]) - S.c0[a];
        if (c < 0 || c >= S.e[a]) return -1;
        l[a] = c;
    }
    return l[0] + S.e[0] * (l[1] + S.e[1] * l[2]);
}

// Full build, part 1: bin the unsorted particles of replica r into per-brick buckets.
__global__ void k_gbin(Buffers B, int64_t S_, int cur, int r)
{
    const RepDev &R = B.reps[r];
    int64_t tg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tg >= R.n) return;
    if (!(B.flags[r] & FLAG_FULL)) return;
    int64_t d = R.p_off + tg;
    int c[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double t = B.x[cur][3 * d + a];
        if (!isfinite(t)) {
            bad = true;
            t = 0.0;
        }
        t = wrap1(t, R.L[a]);
        B.x[cur][3 * d + a] = t;
        c[a] = cell_of(t, R.h[a], R.nc[a]) / R.bd[a];
    }
    if (bad) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NONFINITE);
    int lb = c[0] + R.nb[0] * (c[1] + R.nb[1] * c[2]);
    int idx = atomicAdd(&B.bfill[R.b_off + lb], 1);
    if (idx < R.bcap)
        B.src[R.p_off + (int64_t)lb * R.bcap + idx] = (int32_t)d;
    else
        atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
}

// Full build, part 2: order each bucket and write the next layout.
__global__ void k_gsort(Buffers B, Launch P, int cur)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & FLAG_FULL)) return;
    int lb = b - R.b_off;
    SortTabs T = carve_sort(smem, P.bcap_max, P.ncb_max);
    if (threadIdx.x == 0) {
        brick_geometry(R, lb, S);
        S.rank0 = B.brick_rank0[b];
    }
    __syncthreads();
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) {
        T.hist[lc] = 0;
        T.fill[lc] = 0;
    }
    __syncthreads();
    int nmem = min(B.bfill[b], R.bcap);
    const int64_t S_ = P.nslots;
    for (int m = threadIdx.x; m < nmem; m += blockDim.x) {
        int d = B.src[S.base + m];
        double xw[3] = {B.x[cur][3 * d], B.x[cur][3 * d + 1], B.x[cur][3 * d + 2]};
        int lc = local_cell(R, S, xw);
        if (lc < 0) lc = 0;  // not reached: binned from the same wrapped coordinates
        T.m_src[m] = d;
        T.m_tag[m] = B.tag[d];
        T.m_lc[m] = lc;
        atomicAdd(&T.hist[lc], 1);
    }
    __syncthreads();
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) T.cpre[lc] = T.hist[lc];
    __syncthreads();
    place_members(B, R, r, b, S, T, nmem, cur, S_);
    __syncthreads();
    if (threadIdx.x == 0) B.bfill[b] = 0;
}

// Incremental build: gather the particles now inside the brick from the one-cell halo of
// the current layout (a particle moves less than one cell between builds), order them and
// write the next layout.
__global__ void k_resort(Buffers B, Launch P, int cur)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr Ssh;
    __shared__ int nmem_s;
    int b;
    if (!brick_of_block(P, B, b)) return;
    // replica 0's flags read beside the owner: with one replica (the usual case) the test
    // that ends most launches needs no dependent read
    const uint32_t fl0 = B.flags[0];
    const int r = B.brick_rep[b];
    const int tot = B.stotal[b];
    if (r < 0) return;
    const uint32_t fl = r == 0 ? fl0 : B.flags[r];
    if (!(fl & VBC_FLAG_REBUILD) || (fl & FLAG_FULL)) return;
    // the staging map's first entries are read only once a build is due: a launch on a
    // step without a build (most steps) then reads nothing but the flags
    const MapFirst mf = map_prefetch(B, b, P.stage_cap);
    const RepDev &R = B.reps[r];
    int lb = b - R.b_off;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs Q = carve_tabs(smem, nh_cap);
    SortTabs T = carve_sort(after_tabs(smem, nh_cap), P.bcap_max, P.ncb_max);
    // the candidates (the brick and its one-cell halo in the live layout) are exactly the
    // particles the last list build staged: read them through its staging map (header in
    // every thread, no cell-table walk); after an overflowed build, walk the cell tables
    const bool use_map = tot <= P.stage_cap;
    StageHdr S;
    if (use_map) {
        pass_header(R, B, b, lb, P.stage_cap, S);
        S.rank0 = B.brick_rank0[b];
    } else {
        stage_tables(R, b, lb, B.brick_rank0, B.cell_rank, B.cstart[0], B.ccnt[0], B.bcnt[0], Ssh, Q,
                     1 << 30);
        S = Ssh;
    }
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) {
        T.hist[lc] = 0;
        T.fill[lc] = 0;
    }
    if (threadIdx.x == 0) nmem_s = 0;
    __syncthreads();
    const int64_t S_ = P.nslots;
    const int bcap = R.bcap;
    auto member = [&](int src, bool ok) {
        double xw[3];
        for (int a = 0; a < 3; ++a) xw[a] = wrap1(B.x[cur][3 * src + a], R.L[a]);
        const int tg = B.tag[src];
        int lc = local_cell(R, S, xw);
        if (ok && lc >= 0) {
            int m = atomicAdd(&nmem_s, 1);
            if (m < bcap) {
                T.m_src[m] = src;
                T.m_tag[m] = tg;
                T.m_lc[m] = lc;
                atomicAdd(&T.hist[lc], 1);
            }
        }
    };
    if (use_map) stage_map4(B, b, P.stage_cap, S, mf, [&](int t, int src, int w, bool ok) { member(src, ok); });
    else stage_copy(S, Q, [&](int t, int src, int w) { member(src, true); });
    __syncthreads();
    int nmem = nmem_s;
    if (nmem > bcap) {
        if (threadIdx.x == 0) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
        nmem = bcap;
    }
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) T.cpre[lc] = T.hist[lc];
    __syncthreads();
    place_members(B, R, r, b, S, T, nmem, cur, S_);
}

// ---------------------------------------------------------------------------
// list build, step 2: copy to live, build the list
// ---------------------------------------------------------------------------

// Copy brick b of the next layout into the live arrays and list, for each own particle,
// every staged j != i with minimum-image r^2 < r_list^2.  The decision is exact: the
// staged FP32 brick-local positions decide every pair whose r^2 is further than 1e-4 from
// r_list^2 (their error is below 2e-5), and the remaining pairs are tested with the same
// FP64 expression as the plain definition -- t = x_i - x_j, d = t - L k with k the image
// of the halo cell, r^2 = (dx dx + dy dy) + dz dz, no contraction.  Entries are written
// eight at a time as 16-byte chunks.
//
// The candidate scan reads a second copy of the staged positions in LDS, laid out in the
// x-fastest order of the whole (e+2)^3 cell grid, own and halo cells together: the three
// cells of a stencil row along x are then one contiguous range, and a lane walks 9 ranges
// instead of 27 cells (a wave pays the longest range among its lanes, about 20 % fewer
// iterations).  Entries are the staging-order indices, so the lists are the same.
#ifndef NLIST_ATTR
#define NLIST_ATTR __attribute__((amdgpu_waves_per_eu(6)))
#endif
#ifndef SCAN_UNROLL
#define SCAN_UNROLL 4  // candidate positions read ahead in the list build's scan
#endif
__global__ void NLIST_ATTR k_nlist(Buffers B, Launch P, int cur)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    __shared__ unsigned long long lost_sum, ent_sum;
    __shared__ unsigned pmax_bits;  // largest |p|^2 of the staged positions (FP32 bits)
    int b, r;
    const uint32_t fl0 = B.flags[0];  // as in k_resort
    if (!resolve_brick(P, B, b, r)) return;
    if (!((r == 0 ? fl0 : B.flags[r]) & (VBC_FLAG_REBUILD | FLAG_FULL))) return;
    const RepDev &R = B.reps[r];
    int lb = b - R.b_off;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    float4 *hpos = (float4 *)after_tabs(smem, nh_cap);    // staged positions, grid order
    int *hq = (int *)(hpos + P.stage_cap + SCAN_UNROLL);  // first grid-order index of each cell
    uint16_t *conv = (uint16_t *)(hq + nh_cap + 4);      // grid order -> staging order
    const int64_t S_ = P.nslots;

    if (threadIdx.x == 0) {
        lost_sum = 0ull;
        ent_sum = 0ull;
        pmax_bits = 0u;
    }
    stage_tables(R, b, lb, B.brick_rank0, B.cell_rank, B.cstart[1], B.ccnt[1], B.bcnt[1], S, T,
                 P.stage_cap);

    // next layout -> live for the own range and the own cell tables
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.base + t;
        for (int a = 0; a < 3; ++a) {
            double xa = B.xs[3 * i + a];
            B.x[cur][3 * i + a] = xa;
            B.xref[a * S_ + i] = xa;
            B.v[a * S_ + i] = B.vs[a * S_ + i];
        }
        B.tag[i] = B.tags[i];
        B.type[i] = B.types[i];
        B.lcell[i] = B.lcells[i];
    }
    for (int lc = threadIdx.x; lc < S.ncb; lc += blockDim.x) {
        B.cstart[0][R.c_off + S.rank0 + lc] = B.cstart[1][R.c_off + S.rank0 + lc];
        B.ccnt[0][R.c_off + S.rank0 + lc] = B.ccnt[1][R.c_off + S.rank0 + lc];
    }
    if (threadIdx.x == 0) B.bcnt[0][b] = S.n_own;
    if (lb == 0) {
        // every particle must have been placed in exactly one brick of the next layout
        unsigned long long placed = 0;
        for (int k = threadIdx.x; k < R.nbrick; k += blockDim.x) placed += B.bcnt[1][R.b_off + k];
        placed = wave_sum(placed);
        if ((threadIdx.x % VBC_WAVE) == 0 && placed) atomicAdd(&lost_sum, placed);
        __syncthreads();
        if (threadIdx.x == 0) {
            B.stats[4 * r + 0] += 1ull;
            if (lost_sum != (unsigned long long)R.n) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_LOST);
        }
    }
    if (threadIdx.x == 0) B.stotal[b] = S.total;
    if (S.overflow) {
        for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) B.nn[S.base + t] = 0;
        if (threadIdx.x == 0) {
            atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
            B.bentries[b] = 0u;
        }
        return;
    }
    int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    uint8_t *wm = B.wmap + (size_t)b * P.stage_cap;
    // grid-order offsets: exclusive prefix of every cell's count, the total at hq[nh]
    for (int q = threadIdx.x; q < S.nh; q += blockDim.x) hq[q] = T.q_cnt[q];
    __syncthreads();
    {
        const int tot = wave0_exclusive_scan(hq, S.nh);
        if (threadIdx.x == 0) hq[S.nh] = tot;
    }
    __syncthreads();
    {
        // staging copy (as stage_copy), each particle also placed at its grid-order index
        // with |p|^2 in the fourth component (brick-centred FP32 coordinates)
        const int gid = threadIdx.x / VBC_GROUP, gl = threadIdx.x % VBC_GROUP;
        const int ng = blockDim.x / VBC_GROUP;
        float pm2 = 0.0f;
        for (int q = gid; q < S.nh; q += ng) {
            const int off = T.q_off[q], src0 = T.q_src[q], cnt = T.q_cnt[q], w = T.q_w[q], h0 = hq[q];
            for (int k = gl; k < cnt; k += VBC_GROUP) {
                const int t = off + k, src = src0 + k;
                sm[t] = src;
                wm[t] = (uint8_t)w;
                float4 p;
                p.x = (float)((B.xs[3 * src] + R.L[0] * (double)unpack_w(w, 0)) - S.O[0]);
                p.y = (float)((B.xs[3 * src + 1] + R.L[1] * (double)unpack_w(w, 1)) - S.O[1]);
                p.z = (float)((B.xs[3 * src + 2] + R.L[2] * (double)unpack_w(w, 2)) - S.O[2]);
                p.w = fmaf(p.x, p.x, fmaf(p.y, p.y, p.z * p.z));
                pm2 = fmaxf(pm2, p.w);
                hpos[h0 + k] = p;
                conv[h0 + k] = (uint16_t)t;
            }
        }
#pragma unroll
        for (int o = VBC_WAVE / 2; o > 0; o >>= 1) pm2 = fmaxf(pm2, __shfl_xor(pm2, o, VBC_WAVE));
        if ((threadIdx.x % VBC_WAVE) == 0) atomicMax(&pmax_bits, __float_as_uint(pm2));  // pm2 >= 0
        // the scan reads up to SCAN_UNROLL - 1 records past a row's end: far-away padding
        if ((int)threadIdx.x < SCAN_UNROLL) hpos[S.total + threadIdx.x] = make_float4(1e18f, 1e18f, 1e18f, 3e36f);
    }
    __syncthreads();

    const double rl2 = R.rlist2;
    const float lo2 = (float)(rl2 * (1.0 - 2e-5) - 1e-4), hi2 = (float)(rl2 * (1.0 + 2e-5) + 1e-4);
    // The pre-filter tests d = (|p_u|^2 - c_i) - 2 p_i.p_u < 0 with c_i = hi2 + margin - |p_i|^2:
    // one subtraction and three fused steps per candidate.  With P2 the largest staged |p|^2
    // and u = 2^-24, the rounded squares, the subtractions and the fused steps (whose partial
    // sums stay below 4 P2 + hi2) err by less than 25 u (P2 + hi2) in total, and the direct
    // form |p_i - p_u|^2 that decides the list differs from the exact local distance by at
    // most 5 u hi2; the margin, 128 u (P2 + hi2), is four times their sum.  So every candidate
    // that the direct form puts below hi2 is marked, and every candidate with d + delta < 0,
    // delta = (hi2 + margin) - (lo2 - margin), has the direct form below lo2: such a "sure"
    // candidate is in the list without another test, and the other marked ones are decided
    // as before (direct form against lo2 and hi2, FP64 in between).
    const float P2 = __uint_as_float(pmax_bits), marg = 0x1p-17f * (P2 + hi2);
    const float hi2m = hi2 + marg, delta = hi2m - (lo2 - marg);
    const int kmax = P.k_max;
    // read once: the global descriptor cannot be kept in registers across the list stores
    const int xspan = R.excl_span, cl = R.chain_len;
    bool ovf = false;
    unsigned long long entries = 0;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.base + t;
        const int ta = xspan > 0 ? B.tags[i] : 0;
        int loc = B.lcells[i];
        int lx = loc % S.e[0], ly = (loc / S.e[0]) % S.e[1], lz = loc / (S.e[0] * S.e[1]);
        const int qs = (lx + 1) + S.H[0] * ((ly + 1) + S.H[1] * (lz + 1));
        const int hs = hq[qs] + (t - T.q_off[qs]);  // this particle in grid order
        const float4 pi = hpos[hs];
        const float mx = -2.0f * pi.x, my = -2.0f * pi.y, mz = -2.0f * pi.z, ci = hi2m - pi.w;
        int nn = 0, e = 0;
        // the open chunk as one 128-bit shift register, newest entry in the low half of b0
        uint32_t b0 = 0u, b1 = 0u, b2 = 0u, b3 = 0u;
        uint4 *wp = B.nl + i;  // where the open chunk goes
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy) {
                // the row of three cells along x, one contiguous grid-order range, in segments
                // of 32 candidates: a tight loop marks the candidates that the FP32 pre-filter
                // keeps, then a second loop visits only the marked ones in order, repeats the
                // FP32 test (the few close calls to the list radius are decided in FP64) and
                // appends.  The wave then pays the longest segment among its lanes only for
                // the few instructions of the test, and the append only per neighbour.
                const int q0 = lx + S.H[0] * ((ly + dy) + S.H[1] * (lz + dz));
                const int ub = hq[q0], u1 = hq[q0 + 1], u2 = hq[q0 + 2], ue = hq[q0 + 3];
                for (int u0 = ub; u0 < ue; u0 += 32) {
                    const int n = min(32, ue - u0), cnt = (n + SCAN_UNROLL - 1) & ~(SCAN_UNROLL - 1);
                    // the sign bit of each candidate's d shifted in from the right: candidate k
                    // of the segment ends at bit cnt - 1 - k.  Reads past the row (into its
                    // successors or the padding) are masked below
                    uint32_t near = 0u, sure = 0u;
                    for (int k0 = 0; k0 < n; k0 += SCAN_UNROLL) {
                        const float4 *pp = hpos + (u0 + k0);
                        float4 pu[SCAN_UNROLL];
#pragma unroll
                        for (int j = 0; j < SCAN_UNROLL; ++j) pu[j] = pp[j];
#pragma unroll
                        for (int j = 0; j < SCAN_UNROLL; ++j) {
                            float d = pu[j].w - ci;
                            d = fmaf(pu[j].x, mx, d);
                            d = fmaf(pu[j].y, my, d);
                            d = fmaf(pu[j].z, mz, d);
                            near = __builtin_amdgcn_alignbit(near, __float_as_uint(d), 31);
                            sure = __builtin_amdgcn_alignbit(sure, __float_as_uint(d + delta), 31);
                        }
                    }
                    near &= ~((1u << (cnt - n)) - 1u);
                    if (u0 <= hs && hs < u0 + n) near &= ~(1u << (cnt - 1 - (hs - u0)));  // not itself
                    uint32_t todo = near;
                    while (todo) {
                        const int bit = 31 - __builtin_clz(todo);
                        todo &= ~(1u << bit);
                        const int u = u0 + (cnt - 1 - bit);
                        uint32_t hv = (uint32_t)conv[u];
                        bool in = (sure >> bit) & 1u;
                        if (!in) {
                            const float4 pu = hpos[u];
                            const float ex = pi.x - pu.x, ey = pi.y - pu.y, ez = pi.z - pu.z;
                            const float r2f = ex * ex + ey * ey + ez * ez;
                            in = r2f < lo2;
                            if (!in && r2f < hi2) {
                                // near the list radius: decide with the exact FP64 expression
                                const int q = q0 + (u >= u1 ? 1 : 0) + (u >= u2 ? 1 : 0);
                                const int w = T.q_w[q];
                                int64_t js = T.q_src[q] + (u - hq[q]);
                                double kx = (double)unpack_w(w, 0), ky = (double)unpack_w(w, 1),
                                       kz = (double)unpack_w(w, 2);
                                double r2;
                                {
#pragma clang fp contract(off)
                                    double tx = B.xs[3 * i] - B.xs[3 * js];
                                    double ty = B.xs[3 * i + 1] - B.xs[3 * js + 1];
                                    double tz = B.xs[3 * i + 2] - B.xs[3 * js + 2];
                                    double ddx = tx - R.L[0] * kx;
                                    double ddy = ty - R.L[1] * ky;
                                    double ddz = tz - R.L[2] * kz;
                                    r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
                                }
                                in = r2 < rl2;
                            }
                        }
                        if (in) {
                            if (xspan > 0) {
                                // chain neighbours up to excl_span beads apart: bit 15
                                const int q = q0 + (u >= u1 ? 1 : 0) + (u >= u2 ? 1 : 0);
                                const int tb = B.tags[T.q_src[q] + (u - hq[q])];
                                const int db = ta - tb;
                                if (ta / cl == tb / cl && db <= xspan && -db <= xspan) hv |= 0x8000u;
                            }
                            b3 = __builtin_amdgcn_alignbit(b3, b2, 16);
                            b2 = __builtin_amdgcn_alignbit(b2, b1, 16);
                            b1 = __builtin_amdgcn_alignbit(b1, b0, 16);
                            b0 = (b0 << 16) | hv;
                            ++nn;
                            if (++e == CHUNK) {
                                if (nn <= kmax) *wp = make_uint4(b0, b1, b2, b3);
                                wp += S_;
                                e = 0;
                            }
                        }
                    }
                }
            }
        if (e && nn <= kmax) {
            // pad the last chunk with the dummy staged slot (far away: contributes nothing)
            const uint32_t D = (uint32_t)P.stage_cap;
            for (; e < CHUNK; ++e) {
                b3 = __builtin_amdgcn_alignbit(b3, b2, 16);
                b2 = __builtin_amdgcn_alignbit(b2, b1, 16);
                b1 = __builtin_amdgcn_alignbit(b1, b0, 16);
                b0 = (b0 << 16) | D;
            }
            *wp = make_uint4(b0, b1, b2, b3);
        }
        if (nn > kmax) {
            ovf = true;
            nn = kmax;
        }
        B.nn[i] = (uint16_t)nn;
        entries += (unsigned long long)nn;
    }
    if (ovf) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NLIST_OVERFLOW);
    entries = wave_sum(entries);
    if ((threadIdx.x % VBC_WAVE) == 0 && entries) atomicAdd(&ent_sum, entries);
    __syncthreads();
    if (threadIdx.x == 0) B.bentries[b] = (uint32_t)ent_sum;
}

// ---------------------------------------------------------------------------
// list sweep helper
// ---------------------------------------------------------------------------

// The descriptor of replica r: the launch's own copy for a fixed single replica, else the
// workspace's.
template <bool ONE>
__device__ __forceinline__ const RepDev &rep_of(const OneRep<ONE> &R1, const Buffers &B, int r)
{
    if constexpr (ONE) return R1.R;
    else return B.reps[r];
}

// Visit the list of one own particle in whole chunks of eight entries (the last chunk is
// padded with the dummy staged slot, whose terms all vanish), with the next chunk's load
// issued before the current one is processed.  fn(staged index) is called for every entry
// of a chunk without a guard, so the eight LDS gathers of a chunk can be in flight together.
template <class F>
__device__ __forceinline__ void for_each_neighbour(const uint4 *__restrict__ nl, int64_t S_,
                                                   int64_t i, int nn, F &&fn)
{
    int nch = (nn + CHUNK - 1) / CHUNK;
    if (nch == 0) return;
    const uint4 *lp = nl + i;
    uint4 q = lp[0];
    for (int c = 0; c < nch; ++c) {
        uint4 qn = (c + 1 < nch) ? lp[(size_t)(c + 1) * S_] : q;
        uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < CHUNK; ++e) fn((int)((w[e >> 1] >> (16 * (e & 1))) & 0xffffu));
        q = qn;
    }
}

// The dummy staged slot that pads list chunks: far from every particle of the brick.
template <class R4>
__device__ __forceinline__ R4 dummy_pos()
{
    R4 p;
    p.x = 1.0e6f;
    p.y = 1.0e6f;
    p.z = 1.0e6f;
    p.w = 0;
    return p;
}

// ---------------------------------------------------------------------------
// pass 1: counts
// ---------------------------------------------------------------------------

// Pair constants converted to the pair-arithmetic precision.
template <class Real>
struct PairR {
    Real E_r, c_r, inv_rr2, E_a, c_a, m, inv_w, r_l, inv_dw, c_c, rl2, rh2, rc2;
    Real x1, x2;
    Real k_r;      // -c_r / r_r^2: V_r'(r)/r = c_r + k_r r^2 inside the core
    Real nm_w;     // -m / w:  u_a = r / w + nm_w
    Real nrl_dw;   // -r_l / (r_h - r_l):  u_c = r / (r_h - r_l) + nrl_dw
    int attract;
};

template <class Real>
__device__ __forceinline__ PairR<Real> pair_r(const PairDev &p, double rc2)
{
    PairR<Real> q;
    q.E_r = (Real)p.E_r;
    q.c_r = (Real)p.c_r;
    q.inv_rr2 = (Real)p.inv_rr2;
    q.E_a = (Real)p.E_a;
    q.c_a = (Real)p.c_a;
    q.m = (Real)p.m;
    q.inv_w = (Real)p.inv_w;
    q.r_l = (Real)p.r_l;
    q.inv_dw = (Real)p.inv_dw;
    q.c_c = (Real)p.c_c;
    q.rl2 = (Real)p.rl2;
    q.rh2 = (Real)p.rh2;
    q.rc2 = (Real)rc2;
    q.x1 = (Real)p.x1;
    q.x2 = (Real)p.x2;
    q.k_r = (Real)(-p.c_r * p.inv_rr2);
    q.nm_w = (Real)(-p.m * p.inv_w);
    q.nrl_dw = (Real)(-p.r_l * p.inv_dw);
    q.attract = p.attract;
    return q;
}

// Brick-local position of a staged particle: (x + k L) - O, rounded once to Real.
template <class Real>
__device__ __forceinline__ typename V4<Real>::t local_pos(const RepDev &R, const StageHdr &S,
                                                          const double *__restrict__ X,
                                                          int64_t S_, int src, int w, int type)
{
    typename V4<Real>::t p;
    p.x = (Real)((X[3 * src] + R.L[0] * (double)unpack_w(w, 0)) - S.O[0]);
    p.y = (Real)((X[3 * src + 1] + R.L[1] * (double)unpack_w(w, 1)) - S.O[1]);
    p.z = (Real)((X[3 * src + 2] + R.L[2] * (double)unpack_w(w, 2)) - S.O[2]);
    p.w = (Real)type;
    return p;
}

template <class Real>
__device__ __forceinline__ void load_pairs(const RepDev &R, PairR<Real> *pt)
{
    const int nt = R.ntypes;
    if ((int)threadIdx.x < nt * nt) {
        int a = threadIdx.x / nt, c = threadIdx.x % nt;
        pt[a * MAXT + c] = pair_r<Real>(R.pair[a * MAXT + c], R.rc2);
    }
}

// One term of eq. (counter) in FP64: omega(r, r_l, r_h) = (1 - u^2)^2 with
// u = (r - r_l)/(r_h - r_l), exactly 1 inside r_l and 0 beyond r_h.
__device__ __forceinline__ double count_term64(double r2, const PairDev &p)
{
    if (r2 <= p.rl2) return 1.0;
    if (r2 >= p.rh2) return 0.0;
    const double u = (sqrt(r2) - p.r_l) * p.inv_dw;
    const double q = 1.0 - u * u;
    return q * q;
}

// With FP32 pair arithmetic a particle is listed for an FP64 recount when its FP32 count
// lies within this margin of a switching window (the FP32 count is within about 1e-5 of
// the exact one), so that every particle whose exact count lies inside a window is listed.
constexpr double COUNT_MARGIN = 1e-4;

// Counts in FP64 of the particles the FP32 count pass listed (brick b, its first nw
// entries of wlst): their switching factor s and dU/dn depend steeply on n (eq. (Psi),
// eq. (Psidelta)), so the count is summed again from the FP64 positions, gathered through
// the brick's staging map, instead of the FP32 staged ones (whose rounding would move each
// count term by up to about 3e-6).  A group of LANES lanes per particle: lane l takes list
// entry l % 8 of chunk l / 8 (+ LANES / 8 per further chunk it reads), CP chunks per lane
// in a phase of three dependent gathers (list chunk, staging map, position) that go out
// together; the partial sums are added in a fixed order.  Writes n (FP64), s (or n with
// several types) and, if asked, the caller-order count.
template <class Real, bool MULTI, int LANES, int CP>
__device__ __forceinline__ void recount_window(const Buffers &B, const Launch &P, const RepDev &R, int b,
                               int64_t base, int nw, const double *__restrict__ X,
                               double *__restrict__ n_out)
{
    using R2 = typename V2<Real>::t;
    constexpr int CG = LANES / CHUNK;  // chunks read side by side by one group
    const int g = threadIdx.x / LANES, l = threadIdx.x % LANES, ng = blockDim.x / LANES;
    const int e = l % CHUNK, cl = l / CHUNK;
    const int64_t S_ = P.nslots;
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    const uint8_t *wm = B.wmap + (size_t)b * P.stage_cap;
    const bool xr = R.excl_span > 0;
    const double L0 = R.L[0], L1 = R.L[1], L2 = R.L[2];
    const PairDev p0 = R.pair[0];
    R2 *sA = (R2 *)B.sA;
    for (int k = g; k < nw; k += ng) {
        const int t = B.wlst[base + k];
        const int64_t i = base + t;
        const double xi0 = X[3 * i], xi1 = X[3 * i + 1], xi2 = X[3 * i + 2];
        const int ti = MULTI ? B.type[i] : 0;
        const int nch = (B.nn[i] + CHUNK - 1) / CHUNK;
        double acc = 0.0;
        // no branch between the loads of a phase; rows past the list (every slot has nchunk
        // rows) and the padding slot read valid memory and are masked
        for (int c0 = 0; c0 < nch; c0 += CG * CP) {
            uint4 q[CP];
#pragma unroll
            for (int j = 0; j < CP; ++j) q[j] = B.nl[(size_t)min(c0 + cl + j * CG, P.nchunk - 1) * S_ + i];
            int uj[CP], src[CP], w[CP];
            bool vj[CP];
#pragma unroll
            for (int j = 0; j < CP; ++j) {
                const uint32_t wd = (e < 2) ? q[j].x : (e < 4) ? q[j].y : (e < 6) ? q[j].z : q[j].w;
                int u = (int)((wd >> (16 * (e & 1))) & 0xffffu);
                bool ok = c0 + cl + j * CG < nch;
                if (MULTI && xr) {
                    ok = ok && !(u >> 15);  // excluded pair: not counted
                    u &= 0x7fff;
                }
                vj[j] = ok && u != P.stage_cap;  // padding of the last chunk
                uj[j] = vj[j] ? u : 0;
            }
#pragma unroll
            for (int j = 0; j < CP; ++j) {
                src[j] = sm[uj[j]];
                w[j] = wm[uj[j]];
            }
            double xj[CP][3];
#pragma unroll
            for (int j = 0; j < CP; ++j)
                for (int a = 0; a < 3; ++a) xj[j][a] = X[3 * src[j] + a];
#pragma unroll
            for (int j = 0; j < CP; ++j) {
                const double dx = xi0 - (xj[j][0] + L0 * (double)unpack_w(w[j], 0));
                const double dy = xi1 - (xj[j][1] + L1 * (double)unpack_w(w[j], 1));
                const double dz = xi2 - (xj[j][2] + L2 * (double)unpack_w(w[j], 2));
                const double r2 = (dx * dx + dy * dy) + dz * dz;
                if (MULTI) {
                    const int tj = B.type[src[j]];
                    if (vj[j] && ((R.mask[ti] >> tj) & 1u)) acc += count_term64(r2, R.pair[ti * MAXT + tj]);
                } else {
                    if (vj[j]) acc += count_term64(r2, p0);
                }
            }
        }
#pragma unroll
        for (int o = LANES / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LANES);
        if (l == 0) {
            B.nd[i] = acc;
            sA[i] = R2{MULTI ? (Real)acc : (Real)omega_d64(acc, p0.x1, p0.x2), Real(0)};
            if (n_out) n_out[R.o_off + B.tag[i]] = acc;
        }
    }
}

__device__ __forceinline__ double replica_sum(const Buffers &B, const RepDev &R);
__device__ __forceinline__ void thermo_add(const Buffers &B, const RepDev &R, int r);

// STATS: also count the ordered pairs inside the interaction cutoff (the pair-evaluation
// statistic); the step loop samples it on one step in eight.
template <class Real, bool MULTI, bool STATS, bool ONE>
__global__ void __attribute__((amdgpu_waves_per_eu(8))) k_count(Buffers B, Launch P, int cur, double *__restrict__ n_out, int advance, OneRep<ONE> R1)
{
    using R4 = typename V4<Real>::t;
    using R2 = typename V2<Real>::t;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ int nwin;  // own particles inside a switching window
    __shared__ unsigned long long ev_sum;
    __shared__ PairR<Real> pt[MAXT * MAXT];
    int b;
    if (!brick_of_block(P, B, b)) return;
    const MapFirst mf = map_prefetch(B, b, P.stage_cap);
    // one fixed replica: its descriptor comes with the launch, no owner lookup
    const int r = ONE ? 0 : B.brick_rep[b];
    if (r < 0) return;
    const RepDev &R = rep_of<ONE>(R1, B, r);
    int lb = b - R.b_off;
    if (lb == 0 && threadIdx.x == 0) atomicAnd(&B.flags[r], ~(uint32_t)VBC_FLAG_REBUILD);
    // the replica's first brick adds the energy and virial sums the last time step's force
    // pass left (with the sums on), after its own work
    const int pend = lb == 0 ? B.tpend[r] : 0;
    R4 *spos = (R4 *)smem;
    constexpr bool SOA = !MULTI && sizeof(Real) == 4;
    float2 *sxy = (float2 *)smem;
    float *sza = (float *)(sxy + P.stage_cap + 1);
    const int64_t S_ = P.nslots;
    load_pairs<Real>(R, pt);
    if (threadIdx.x == 0) {
        nwin = 0;
        ev_sum = 0ull;
    }
    // every thread reads the header itself (uniform values), so that the staging gathers
    // need not wait for a barrier; the staging barrier orders pt, nwin and ev_sum
    StageHdr S;
    pass_header(R, B, b, lb, P.stage_cap, S);
    R2 *sA = (R2 *)B.sA;
    if (S.overflow) {
        for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
            int64_t i = S.base + t;
            B.nd[i] = 0.0;
            sA[i] = R2{Real(0), Real(0)};
        }
        if (threadIdx.x == 0) {
            atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
            B.wcnt[b] = 0;
        }
        if (pend) thermo_add(B, R, r);
        return;
    }
    const double *X = B.x[cur];
    stage_map4(B, b, P.stage_cap, S, mf, [&](int t, int src, int w, bool ok) {
        const R4 p = local_pos<Real>(R, S, X, S_, src, w, MULTI ? B.type[src] : 0);
        if (ok) {
            if (SOA) {
                sxy[t] = make_float2((float)p.x, (float)p.y);
                sza[t] = (float)p.z;
            } else {
                spos[t] = p;
            }
        }
    });
    if (threadIdx.x == 0) {
        if (SOA) {
            sxy[P.stage_cap] = make_float2(1.0e6f, 1.0e6f);
            sza[P.stage_cap] = 1.0e6f;
        } else {
            spos[P.stage_cap] = dummy_pos<R4>();
        }
    }
    __syncthreads();

    const PairR<Real> p0 = pt[0];
    const bool xr = R.excl_span > 0;  // list entries carry the exclusion bit 15
    // read once: the global descriptor cannot be kept in registers across the stores below
    const double wx1 = R.pair[0].x1, wx2 = R.pair[0].x2;
    const bool watt = R.pair[0].attract;
    const int64_t o_off = R.o_off;
    unsigned long long evals = 0;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.base + t;
        R4 pi;
        if (SOA) {
            const float2 q = sxy[t];
            pi.x = q.x;
            pi.y = q.y;
            pi.z = sza[t];
            pi.w = 0;
        } else {
            pi = spos[t];
        }
        int ti = MULTI ? (int)pi.w : 0;
        int inside = 0;
        double n = 0.0;
        Real chunk = Real(0);
        int e = 0;
        // omega(r, r_l, r_h) = (1 - u^2)^2 with u = clamp((r - r_l)/(r_h - r_l), 0, 1): exactly 1
        // inside r_l and 0 beyond r_h; partial sums of eight terms are added in FP64
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            int ex = 0;  // pair excluded from counting and attraction (chain neighbours)
            if (MULTI && xr) {
                ex = u >> 15;
                u &= 0x7fff;
            }
            R4 pj;
            if (SOA) {
                const float2 q = sxy[u];
                pj.x = q.x;
                pj.y = q.y;
                pj.z = sza[u];
                pj.w = 0;
            } else {
                pj = spos[u];
            }
            Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            Real r2 = dx * dx + dy * dy + dz * dz;
            if (STATS) inside += (r2 < p0.rc2) ? 1 : 0;
            Real rr = sqrt_r(r2);
            if (MULTI) {
                int tj = (int)pj.w;
                const PairR<Real> &q = pt[ti * MAXT + tj];
                Real uu = clamp01((rr - q.r_l) * q.inv_dw);
                Real qq = Real(1) - uu * uu;
                chunk += (((R.mask[ti] >> tj) & 1u) && !ex) ? qq * qq : Real(0);
            } else {
                Real uu = clamp01(fma(rr, p0.inv_dw, p0.nrl_dw));
                Real qq = fma(-uu, uu, Real(1));
                chunk = fma(qq, qq, chunk);
            }
            if (++e == CHUNK) {
                n += (double)chunk;
                chunk = Real(0);
                e = 0;
            }
        });
        evals += (unsigned long long)inside;
        B.nd[i] = n;
        bool win = false;
        // with FP32 pair arithmetic the window is widened by the margin: the particles
        // listed get their counts again in FP64 below, before anything reads them
        const double mg = sizeof(Real) == 4 ? COUNT_MARGIN : 0.0;
        if (MULTI) {
            // the switching factor depends on the pair: keep the count itself
            sA[i] = R2{(Real)n, Real(0)};
            for (int u = 0; u < R.ntypes; ++u) {
                const PairDev &pd = R.pair[ti * MAXT + u];
                if (pd.attract && n > pd.x1 - mg && n < pd.x2 + mg) win = true;
            }
        } else {
            sA[i] = R2{(Real)omega_d64(n, wx1, wx2), Real(0)};
            win = watt && n > wx1 - mg && n < wx2 + mg;
        }
        // the dU/dn pass visits only these: list them compactly in the brick's slots
        if (win) B.wlst[S.base + atomicAdd(&nwin, 1)] = (uint16_t)t;
        if (n_out) n_out[o_off + B.tag[i]] = n;
    }
    if (STATS) {
        evals = wave_sum(evals);
        if ((threadIdx.x % VBC_WAVE) == 0 && evals) atomicAdd(&ev_sum, evals);
    }
    __syncthreads();
    if (sizeof(Real) == 4) {
        // the listed entries are in global memory, written by this workgroup before the barrier
        const int nwv = nwin;
        // as many lanes per listed particle (32, 16 or 8) as one round of the workgroup
        // allows: 32 take a list of up to 32 entries in one phase, 16 in two, 8 in four
        if (nwv > 0 && nwv * 32 <= (int)blockDim.x)
            recount_window<Real, MULTI, 32, 1>(B, P, R, b, S.base, nwv, X, n_out);
        else if (nwv > 0 && nwv * 16 <= (int)blockDim.x)
            recount_window<Real, MULTI, 16, 1>(B, P, R, b, S.base, nwv, X, n_out);
        else if (nwv > 0)
            recount_window<Real, MULTI, CHUNK, 1>(B, P, R, b, S.base, nwv, X, n_out);
    }
    if (threadIdx.x == 0) {
        B.wcnt[b] = nwin;
        if (STATS) B.bevals[b] += ev_sum;  // this workgroup is the only writer of brick b
        if (lb == 0) {
            if (STATS) B.stats[4 * r + 3] += 1ull;
            // in a time step the count pass opens the step: the step counter (the noise
            // counter of the Langevin O-step that the following force pass starts) advances
            if (advance) B.step[r] += 1ull;
        }
    }
    if (pend) thermo_add(B, R, r);
}

// ---------------------------------------------------------------------------
// pass 2a: dU/dn for particles inside a switching window
// ---------------------------------------------------------------------------

// Waves per workgroup of the dU/dn pass; one workgroup per brick.
constexpr int EMBED_WAVES = 4;

// dU/dn of the window particles of brick b that fall to group g of ng groups of LPP lanes
// (particles g, g + ng, ...; see k_embed).  t_first: the first particle of this lane's
// group if already read, else -1.
template <int LPP, class Real, bool MULTI>
__device__ __forceinline__ void embed_brick(const Buffers &B, const Launch &P, const RepDev &R,
                                            const PairR<Real> *pt, int b, int64_t base, int nw,
                                            int lane, int g, int ng, int t_first, int cur)
{
    // LPP lanes per window particle, EP entries of each list chunk per lane; neighbours are
    // gathered from global memory through the brick's staging map
    using R2 = typename V2<Real>::t;
    constexpr int EP = CHUNK / LPP;
    const int64_t S_ = P.nslots;
    R2 *sA = (R2 *)B.sA;
    const double *X = B.x[cur];
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    const uint8_t *wm = B.wmap + (size_t)b * P.stage_cap;
    const PairR<Real> p0 = pair_r<Real>(R.pair[0], R.rc2);
    const int e = lane % LPP;
    for (int k = g; k < nw; k += ng) {
        int t = (k == g && t_first >= 0) ? t_first : B.wlst[base + k];
        int64_t i = base + t;
        double n_i = B.nd[i];
        int ti = MULTI ? B.type[i] : 0;
        const double xi0 = X[3 * i], xi1 = X[3 * i + 1], xi2 = X[3 * i + 2];
        int nch = (B.nn[i] + CHUNK - 1) / CHUNK;
        double acc = 0.0;
        if (!MULTI) {
            // four chunks at a time in phases (chunk words, staging map, positions, terms)
            // with no branch between the loads, so that the gathers of all four go out together;
            // rows past the list and the padding slot read valid memory and are masked.  The
            // first four rows are read before the list length arrives (rows below nchunk exist
            // for every slot).
            constexpr int CP = 4 / EP;  // chunks per phase
            uint4 qf[CP];
#pragma unroll
            for (int j = 0; j < CP; ++j) qf[j] = B.nl[(size_t)min(j, P.nchunk - 1) * S_ + i];
            for (int c0 = 0; c0 < nch; c0 += CP) {
                int uj[4], sj[4], wj[4];
                bool vj[4];
                uint4 qc[CP];
#pragma unroll
                for (int j = 0; j < CP; ++j)
                    qc[j] = c0 == 0 ? qf[j] : B.nl[(size_t)min(c0 + j, P.nchunk - 1) * S_ + i];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int jc = j / EP, x = e + LPP * (j % EP);  // chunk, entry
                    const uint4 q = qc[jc];
                    const uint32_t wd = (x < 2) ? q.x : (x < 4) ? q.y : (x < 6) ? q.z : q.w;
                    const int u = (int)((wd >> (16 * (x & 1))) & 0xffffu);
                    vj[j] = c0 + jc < nch && u != P.stage_cap;
                    uj[j] = vj[j] ? u : 0;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sj[j] = sm[uj[j]];
                    wj[j] = wm[uj[j]];
                }
                double xj[4][3];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    for (int a = 0; a < 3; ++a) xj[j][a] = X[3 * sj[j] + a];
                Real sjv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) sjv[j] = sA[sj[j]].x;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    Real dx = (Real)(xi0 - (xj[j][0] + R.L[0] * (double)unpack_w(wj[j], 0)));
                    Real dy = (Real)(xi1 - (xj[j][1] + R.L[1] * (double)unpack_w(wj[j], 1)));
                    Real dz = (Real)(xi2 - (xj[j][2] + R.L[2] * (double)unpack_w(wj[j], 2)));
                    Real r2 = dx * dx + dy * dy + dz * dz;
                    Real uu = (sqrt_r(r2) - p0.m) * p0.inv_w;
                    Real qq = Real(1) - uu * uu;
                    if (vj[j] && qq > Real(0)) acc += (double)(sjv[j] * (-p0.E_a * qq * qq));
                }
            }
        } else {
            for (int cx = 0; cx < nch * EP; ++cx) {
                const int c = cx / EP, x = e + LPP * (cx % EP);
                uint4 q = B.nl[(size_t)c * S_ + i];
                uint32_t wd = (x < 2) ? q.x : (x < 4) ? q.y : (x < 6) ? q.z : q.w;
                int u = (int)((wd >> (16 * (x & 1))) & 0xffffu);
                if (R.excl_span > 0) {
                    if (u & 0x8000) continue;  // excluded pair: no attraction between them
                }
                if (u == P.stage_cap) continue;  // padding
                int src = sm[u], w = wm[u];
                Real dx = (Real)(xi0 - (X[3 * src] + R.L[0] * (double)unpack_w(w, 0)));
                Real dy = (Real)(xi1 - (X[3 * src + 1] + R.L[1] * (double)unpack_w(w, 1)));
                Real dz = (Real)(xi2 - (X[3 * src + 2] + R.L[2] * (double)unpack_w(w, 2)));
                Real r2 = dx * dx + dy * dy + dz * dz;
                int tj = B.type[src];
                const PairR<Real> &q2 = pt[ti * MAXT + tj];
                if (!q2.attract) continue;
                Real uu = (sqrt_r(r2) - q2.m) * q2.inv_w;
                Real qq = Real(1) - uu * uu;
                if (!(qq > Real(0))) continue;
                const PairDev &pd = R.pair[ti * MAXT + tj];
                double sdi = omega_dd64(n_i, pd.x1, pd.x2);
                Real sj = omega_r<Real>(sA[src].x, q2.x1, q2.x2);
                acc += sdi * (double)(sj * (-q2.E_a * qq * qq));
            }
        }
        // fixed-order reduction over the lanes of the group
#pragma unroll
        for (int o = LPP / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LPP);
        if (e == 0) {
            double A = MULTI ? acc : omega_dd64(n_i, R.pair[0].x1, R.pair[0].x2) * acc;
            sA[i].y = (Real)A;
        }
    }
}

// One workgroup of EMBED_WAVES waves per brick over the particles that the count pass
// listed as inside a switching window; most bricks hold a handful or none, and then only
// the first wave works.  No workgroup-wide synchronisation.
template <class Real, bool MULTI>
__global__ void k_embed(Buffers B, Launch P, int cur)
{
    __shared__ PairR<Real> ptab[EMBED_WAVES][MAXT * MAXT];
    const int wv = threadIdx.x / VBC_WAVE, lane = threadIdx.x % VBC_WAVE;
    int b;
    if (!brick_of_block(P, B, b)) return;
    // the brick's owner, window count and staged count read together: most bricks have no
    // window particle and leave here; then the replica descriptor and the first window entry
    const int r = B.brick_rep[b];
    const int nw = B.wcnt[b];
    const int tot = B.stotal[b];
    // free brick, nothing in a window, or an overflowed brick
    if (r < 0 || nw == 0 || tot > P.stage_cap) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    const int64_t base = R.p_off + (int64_t)lb * R.bcap;
    const int t_first = B.wlst[base + lane / CHUNK];  // for eight lanes per particle
    // eight lanes per particle when the first wave takes all of the brick's window particles
    // at once; up to EMBED_WAVES x 8 of them, eight lanes each over every wave; with more,
    // four lanes each over every wave, so that up to EMBED_WAVES x 16 are in flight
    const bool one = nw <= VBC_WAVE / CHUNK;
    if (one && wv > 0) return;
    PairR<Real> *pt = ptab[wv];
    if (MULTI) {
        const int nt = R.ntypes;
        if (lane < nt * nt) {
            const int a = lane / nt, c = lane % nt;
            pt[a * MAXT + c] = pair_r<Real>(R.pair[a * MAXT + c], R.rc2);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (one) {
        embed_brick<CHUNK, Real, MULTI>(B, P, R, pt, b, base, nw, lane, lane / CHUNK, VBC_WAVE / CHUNK,
                                        t_first, cur);
    } else if (nw <= EMBED_WAVES * (VBC_WAVE / CHUNK)) {
        // up to 32: eight lanes each over every wave, all of them in one round
        constexpr int G = VBC_WAVE / CHUNK;
        embed_brick<CHUNK, Real, MULTI>(B, P, R, pt, b, base, nw, lane, wv * G + lane / CHUNK,
                                        EMBED_WAVES * G, -1, cur);
    } else {
        constexpr int G = VBC_WAVE / 4;  // groups of four lanes per wave
        embed_brick<4, Real, MULTI>(B, P, R, pt, b, base, nw, lane, wv * G + lane / 4, EMBED_WAVES * G,
                                    -1, cur);
    }
}

// ---------------------------------------------------------------------------
// pass 2b: forces, energies, virial, fused integration
// ---------------------------------------------------------------------------

// Velocity / position update of one particle, in the same order of operations as the
// plain integrator (no contraction): closing half-kick of the previous step, then the
// opening half-kick and the drift of the next one.
__device__ __forceinline__ void integrate_one(const StepArgs &st, int mode, bool first_kick,
                                              const double F[3], double v[3], double x[3],
                                              uint64_t seed, uint64_t tag, uint64_t step)
{
#pragma clang fp contract(off)
    if (!first_kick)
        for (int a = 0; a < 3; ++a) v[a] = v[a] + st.hdt * F[a];
    if (mode == MODE_LAST) return;
    for (int a = 0; a < 3; ++a) v[a] = v[a] + st.hdt * F[a];
    if (st.kind == VBC_NVE) {
        for (int a = 0; a < 3; ++a) x[a] = x[a] + st.dt * v[a];
    } else {
        for (int a = 0; a < 3; ++a) x[a] = x[a] + st.hdt * v[a];
        double xi[3];
        langevin_noise(seed, tag, step, xi);
        for (int a = 0; a < 3; ++a) v[a] = st.c1 * v[a] + st.c2s * xi[a];
        for (int a = 0; a < 3; ++a) x[a] = x[a] + st.hdt * v[a];
    }
}

template <class Real, bool MULTI, bool THERMO, bool ONE>
__global__ void k_force(Buffers B, Launch P, int cur, int mode, StepArgs st,
                        double *__restrict__ F_out, double *__restrict__ e_out, OneRep<ONE> R1)
{
    using R4 = typename V4<Real>::t;
    using R2 = typename V2<Real>::t;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ PairR<Real> pt[MAXT * MAXT];
    __shared__ double red[8][1024 / VBC_WAVE];
    __shared__ int moved;
    int b;
    if (!brick_of_block(P, B, b)) return;
    const MapFirst mf = map_prefetch(B, b, P.stage_cap);
    const int r = ONE ? 0 : B.brick_rep[b];
    if (r < 0) return;
    const RepDev &R = rep_of<ONE>(R1, B, r);
    int lb = b - R.b_off;
    // staged per particle: position and, with one type, the switching factor s in .w plus
    // c_c A in a separate array (20 bytes in FP32); with several types the type in .w and
    // (s or n, A) beside it
    R4 *spos = (R4 *)smem;
    R2 *ssa = (R2 *)(spos + P.stage_cap + 1);
    Real *scA = (Real *)(spos + P.stage_cap + 1);
    const int64_t S_ = P.nslots;
    const int64_t ntot = P.ntot;
    load_pairs<Real>(R, pt);
    if (threadIdx.x == 0) moved = 0;
    // every thread reads the header itself (as in the count pass); the staging barrier
    // orders pt and moved
    StageHdr S;
    pass_header(R, B, b, lb, P.stage_cap, S);
    const R2 *sA = (const R2 *)B.sA;
    if (S.overflow) {
        if (threadIdx.x == 0) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
        if (THERMO && threadIdx.x < 8) B.part[(size_t)b * 8 + threadIdx.x] = 0.0;
        if (THERMO && st.acc && lb == 0 && threadIdx.x == 0) B.tpend[r] = 1;
        return;
    }
    const double *X = B.x[cur];
    const Real cc0 = pair_r<Real>(R.pair[0], R.rc2).c_c;
    stage_map4(B, b, P.stage_cap, S, mf, [&](int t, int src, int w, bool ok) {
        R4 p = local_pos<Real>(R, S, X, S_, src, w, MULTI ? B.type[src] : 0);
        const R2 sa = sA[src];
        if (!MULTI) p.w = sa.x;
        if (ok) {
            spos[t] = p;
            if (MULTI) ssa[t] = sa;
            else scA[t] = sa.y * cc0;  // one type: the chain-rule term needs only c_c A
        }
    });
    if (threadIdx.x == 0) {
        spos[P.stage_cap] = dummy_pos<R4>();
        if (MULTI) ssa[P.stage_cap] = R2{Real(0), Real(0)};
        else scA[P.stage_cap] = Real(0);
    }
    __syncthreads();

    const PairR<Real> p0 = pt[0];
    const bool xr = R.excl_span > 0;  // list entries carry the exclusion bit 15
    // read once: the global descriptor cannot be kept in registers across the stores below
    const int chain_len = R.chain_len;
    const double disp2 = R.disp2;
    const int64_t o_off = R.o_off;
    const uint64_t step = B.step[r];
    const uint64_t key = st.seed + R.seed;
    // e, -, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz; the scalar virial W is the trace, formed per brick
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool bad = false, mv = false;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.base + t;
        R4 pi = spos[t];
        const R2 sai = MULTI ? ssa[t] : R2{pi.w, scA[t]};
        int ti = MULTI ? (int)pi.w : 0;
        const Real cai = p0.c_a * sai.x;
        // ei: pair energies (several types), or with one type sum tc^2 and ea sum s_j q_a^2,
        // which E_r and E_a s_i scale once per particle
        Real fx = 0, fy = 0, fz = 0, ei = 0, ea = 0;
        Real wxx = 0, wyy = 0, wzz = 0, wxy = 0, wxz = 0, wyz = 0;
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            int ex = 0;  // pair excluded from counting and attraction (chain neighbours)
            if (MULTI && xr) {
                ex = u >> 15;
                u &= 0x7fff;
            }
            R4 pj = spos[u];
            Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            Real r2 = dx * dx + dy * dy + dz * dz;
            Real phr, ep;
            if (MULTI) {
                int tj = (int)pj.w;
                const PairR<Real> &q = pt[ti * MAXT + tj];
                if (!(r2 < q.rc2)) return;
                R2 saj = ssa[u];
                Real rinv = rsqrt_r(r2 > Real(1e-30) ? r2 : Real(1e-30));
                Real rr = r2 * rinv;
                Real tc = Real(1) - r2 * q.inv_rr2;
                tc = tc > Real(0) ? tc : Real(0);
                phr = q.c_r * tc;
                ep = q.E_r * tc * tc;
                if (q.attract && !ex) {
                    Real uu = (rr - q.m) * q.inv_w;
                    Real qq = Real(1) - uu * uu;
                    if (qq > Real(0)) {
                        Real psi = omega_r<Real>(sai.x, q.x1, q.x2) * omega_r<Real>(saj.x, q.x1, q.x2);
                        ep -= q.E_a * psi * qq * qq;
                        phr += psi * q.c_a * uu * qq * rinv;
                    }
                }
                Real asum = ex ? Real(0)
                               : (((R.mask[ti] >> tj) & 1u) ? sai.y : Real(0)) +
                                     (((R.mask[tj] >> ti) & 1u) ? saj.y : Real(0));
                Real uc = (rr - q.r_l) * q.inv_dw;
                uc = uc < Real(0) ? Real(0) : (uc > Real(1) ? Real(1) : uc);
                phr += asum * q.c_c * uc * (Real(1) - uc * uc) * rinv;
            } else {
                // branch-free: beyond every cutoff (and for the padding slot) all three terms
                // vanish through the clamps.  phi/r = min(c_r + k_r r^2, 0)
                //   + [ c_a s_i s_j u_a q_a + (c_c A_i + c_c A_j) u_c (1 - u_c^2) ] / r
                const Real sj = pj.w, cAj = scA[u];
                Real rinv = rsqrt_r(r2 > Real(1e-30) ? r2 : Real(1e-30));
                Real rr = r2 * rinv;
                Real pr = fmin(fma(r2, p0.k_r, p0.c_r), Real(0));
                Real uu = fma(rr, p0.inv_w, p0.nm_w);
                Real qq = fmax(fma(-uu, uu, Real(1)), Real(0));
                Real uc = clamp01(fma(rr, p0.inv_dw, p0.nrl_dw));
                Real g = uc * fma(-uc, uc, Real(1));
                Real t = fma(sai.y + cAj, g, cai * sj * uu * qq);
                phr = fma(t, rinv, pr);
                if (THERMO) {
                    const Real tc = fmax(fma(-r2, p0.inv_rr2, Real(1)), Real(0));
                    ei = fma(tc, tc, ei);
                    ea = fma(sj * qq, qq, ea);
                }
            }
            fx -= phr * dx;
            fy -= phr * dy;
            fz -= phr * dz;
            if (THERMO) {
                if (MULTI) ei += ep;
                wxx -= phr * dx * dx;
                wyy -= phr * dy * dy;
                wzz -= phr * dz * dz;
                wxy -= phr * dx * dy;
                wxz -= phr * dx * dz;
                wyz -= phr * dy * dz;
            }
        });
        double F[3] = {(double)fx, (double)fy, (double)fz};
        double eb = 0.0, wb[7] = {0, 0, 0, 0, 0, 0, 0};
        double xi_[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
        int32_t tg = B.tag[i];
        if (chain_len > 1) {
            // harmonic bonds to the neighbouring beads of the same chain
            int bead = tg % chain_len;
            for (int side = -1; side <= 1; side += 2) {
                if ((side < 0 && bead == 0) || (side > 0 && bead == chain_len - 1)) continue;
                int64_t j = B.inv[o_off + tg + side];
                double d[3];
                for (int a = 0; a < 3; ++a) {
                    double tt = xi_[a] - X[3 * j + a];
                    d[a] = tt - R.L[a] * rint(tt / R.L[a]);
                }
                double rb = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                double dr = rb - R.r0_bond;
                double cf = rb > 0.0 ? R.k_bond * dr / rb : 0.0;
                for (int a = 0; a < 3; ++a) F[a] -= cf * d[a];
                if (THERMO) {
                    eb += 0.25 * R.k_bond * dr * dr;
                    wb[0] -= 0.5 * cf * rb * rb;
                    wb[1] -= 0.5 * cf * d[0] * d[0];
                    wb[2] -= 0.5 * cf * d[1] * d[1];
                    wb[3] -= 0.5 * cf * d[2] * d[2];
                    wb[4] -= 0.5 * cf * d[0] * d[1];
                    wb[5] -= 0.5 * cf * d[0] * d[2];
                    wb[6] -= 0.5 * cf * d[1] * d[2];
                }
            }
        }
        if (!(isfinite(F[0]) && isfinite(F[1]) && isfinite(F[2]))) bad = true;
        if (THERMO) {
            const Real e_pair = MULTI ? ei : p0.E_r * ei - p0.E_a * sai.x * ea;
            double e_i = 0.5 * (double)e_pair + eb;
            acc[0] += e_i;
            acc[2] += 0.5 * (double)wxx + wb[1];
            acc[3] += 0.5 * (double)wyy + wb[2];
            acc[4] += 0.5 * (double)wzz + wb[3];
            acc[5] += 0.5 * (double)wxy + wb[4];
            acc[6] += 0.5 * (double)wxz + wb[5];
            acc[7] += 0.5 * (double)wyz + wb[6];
            if (e_out) e_out[o_off + tg] = e_i;
        }
        if (mode == MODE_EVAL) {
            for (int a = 0; a < 3; ++a) B.Fst[a * S_ + i] = F[a];
            if (F_out)
                for (int a = 0; a < 3; ++a) F_out[a * ntot + o_off + tg] = F[a];
        } else {
            double vv[3] = {B.v[i], B.v[S_ + i], B.v[2 * S_ + i]};
            double xx[3] = {xi_[0], xi_[1], xi_[2]};
            integrate_one(st, mode, false, F, vv, xx, key, (uint64_t)tg, step);
            for (int a = 0; a < 3; ++a) B.v[a * S_ + i] = vv[a];
            if (mode == MODE_LAST) {
                for (int a = 0; a < 3; ++a) B.Fst[a * S_ + i] = F[a];
            } else {
                double *Xn = B.x[cur ^ 1];
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    Xn[3 * i + a] = xx[a];
                    double dd = xx[a] - B.xref[a * S_ + i];
                    d2 += dd * dd;
                }
                if (d2 > disp2) mv = true;
            }
        }
    }
    if (bad) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NONFINITE);
    if (mv) moved = 1;
    if (THERMO) {
        int wv = threadIdx.x / VBC_WAVE, ln = threadIdx.x % VBC_WAVE;
        const double v = wave_sum8(acc);
        if ((ln & 7) == 0) red[ln >> 3][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0 && moved) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_REBUILD);
    if (THERMO && threadIdx.x < 8) {
        int nw = blockDim.x / VBC_WAVE;
        double s = 0.0;
        if (threadIdx.x == 1) {
            // W = W_xx + W_yy + W_zz, summed per wave in the same fixed order
            for (int w = 0; w < nw; ++w) s += (red[2][w] + red[3][w]) + red[4][w];
        } else {
            for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        }
        B.part[(size_t)b * 8 + threadIdx.x] = s;
        // a time step's sums: added by the next count pass or the call's closing reduction
        if (st.acc && lb == 0 && threadIdx.x == 0) B.tpend[r] = 1;
    }
}

// Opening half-kick and drift of the first step of a call, from the forces kept in Fst;
// one workgroup per brick.
__global__ void k_kick_drift(Buffers B, Launch P, int cur, StepArgs st)
{
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int64_t S_ = P.nslots;
    const int64_t base = R.p_off + (int64_t)(b - R.b_off) * R.bcap;
    const int nown = B.bcnt[0][b];
    const uint64_t key = st.seed + R.seed, step = B.step[r];
    bool far = false;
    for (int t = threadIdx.x; t < nown; t += blockDim.x) {
        int64_t i = base + t;
        double F[3], v[3], x[3];
        for (int a = 0; a < 3; ++a) {
            F[a] = B.Fst[a * S_ + i];
            v[a] = B.v[a * S_ + i];
            x[a] = B.x[cur][3 * i + a];
        }
        integrate_one(st, MODE_MID, true, F, v, x, key, (uint64_t)B.tag[i], step);
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            B.v[a * S_ + i] = v[a];
            B.x[cur ^ 1][3 * i + a] = x[a];
            double dd = x[a] - B.xref[a * S_ + i];
            d2 += dd * dd;
        }
        far = far || d2 > R.disp2;
    }
    if (__syncthreads_or(far) && threadIdx.x == 0)
        atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_REBUILD);
}

// Sum of the per-brick energy/virial partial sums of replica R over its bricks, in a fixed
// order (strided per thread, then waves, then the wave totals in order); the result is
// valid in threads 0..7 (one component each).
// The eight sums of replica R's per-brick partial sums, in an order that does not depend on
// the workgroup's size (the count pass and the closing reduction run it with different
// sizes): lane l of the first wave adds bricks l, l + 64, ..., then the wave's lanes are
// added in the fixed order of wave_sum.  Called by the whole workgroup; thread k < 8 gets
// component k.
__device__ __forceinline__ double replica_sum(const Buffers &B, const RepDev &R)
{
    __shared__ double red[8];
    if (threadIdx.x < VBC_WAVE) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = threadIdx.x; b < R.nbrick; b += VBC_WAVE)
            for (int k = 0; k < 8; ++k) acc[k] += B.part[(size_t)(R.b_off + b) * 8 + k];
        for (int k = 0; k < 8; ++k) {
            const double v = wave_sum(acc[k]);
            if (threadIdx.x == 0) red[k] = v;
        }
    }
    __syncthreads();
    return threadIdx.x < 8 ? red[threadIdx.x] : 0.0;
}

// Per-replica totals from the per-brick partial sums, in brick order.
__global__ void k_reduce(Buffers B, int nrep, double *__restrict__ UW)
{
    int r = blockIdx.x;
    const RepDev &R = B.reps[r];
    const double s = replica_sum(B, R);
    if (threadIdx.x < 8) UW[r * 8 + threadIdx.x] = s;
}

// A time step's energy and virial of replica r (kept as the last step's) added to its
// running sums from the per-brick sums its force pass left, and its step count raised by
// one; the pending mark cleared.  Called by a whole workgroup.
__device__ __forceinline__ void thermo_add(const Buffers &B, const RepDev &R, int r)
{
    const double s = replica_sum(B, R);
    if (threadIdx.x < 8) {
        double *T = B.thermo + (size_t)r * THERMO_WORDS;
        T[1 + threadIdx.x] = s;
        T[9 + threadIdx.x] += s;
        if (threadIdx.x == 0) {
            T[0] += 1.0;
            B.tpend[r] = 0;
        }
    }
}

// At the end of a call with the sums on: the last step's sums of every replica with sums
// pending (a slot is live when its first brick is owned by it; retired descriptors stay
// behind).
__global__ void k_thermo_acc(Buffers B, int nrep)
{
    const int r = blockIdx.x;
    const RepDev &R = B.reps[r];
    if (!B.tpend[r]) return;
    if (R.nbrick <= 0 || B.brick_rep[R.b_off] != r) {
        if (threadIdx.x == 0) B.tpend[r] = 0;
        return;
    }
    thermo_add(B, R, r);
}

__global__ void k_thermo_clear(Buffers B, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        B.thermo[i] = 0.0;
        if (i < n / THERMO_WORDS) B.tpend[i] = 0;
    }
}

// Export the list of one replica as tag pairs (inspection and tests).
__global__ void k_export_nlist(Buffers B, Launch P, int rep, int32_t *__restrict__ pairs,
                               int64_t cap, unsigned long long *__restrict__ count)
{
    __shared__ StageHdr S;
    const RepDev &R = B.reps[rep];
    int lb = blockIdx.x;
    if (lb >= R.nbrick) return;
    int b = R.b_off + lb;
    if (threadIdx.x == 0) pass_header(R, B, b, lb, P.stage_cap, S);
    __syncthreads();
    if (S.overflow) return;
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.base + t;
        for_each_neighbour(B.nl, P.nslots, i, B.nn[i], [&](int u) {
            if (R.excl_span > 0) u &= 0x7fff;
            if (u == P.stage_cap) return;  // padding
            unsigned long long k = atomicAdd(count, 1ull);
            if ((int64_t)k < cap) {
                pairs[2 * k] = B.tag[i];
                pairs[2 * k + 1] = B.tag[sm[u]];
            }
        });
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

__global__ void k_zero_i64(int64_t *p, int n)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0;
}

// Squared minimum-image distance from the wrapped position wi of a particle to slot j, in
// FP64 with the operations of the plain definition (round-half-even image, no contraction):
// the bond criterion of the observables and of the cluster analysis.
// Both positions lie in [0, L), so |t| < L and the image index rint(t / L) is -1, 0 or 1;
// away from |t| = L / 2 the comparison t > L / 2 decides it exactly (the quotient is then
// far from 1/2), and only that band takes the division.
__device__ __forceinline__ double obs_r2(const RepDev &R, const double *__restrict__ X, int64_t S_,
                                         const double wi[3], int64_t j)
{
#pragma clang fp contract(off)
    double d[3];
    for (int a = 0; a < 3; ++a) {
        const double La = R.L[a];
        const double tt = wi[a] - wrap1(X[3 * j + a], La);
        const double at = fabs(tt);
        double k;
        if (at < 0.375 * La) k = 0.0;
        else if (at > 0.625 * La) k = tt > 0.0 ? 1.0 : -1.0;
        else k = rint(tt / La);
        d[a] = tt - La * k;
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

// Brick-local FP32 positions (type in w) of every particle the brick staged at the last
// list build, and the dummy slot far away; optionally their slots.  All threads call this.
__device__ __forceinline__ void stage_bonds(const Buffers &B, const Launch &P, const RepDev &R,
                                            const StageHdr &S, int b, const double *X, float4 *spos,
                                            int32_t *ssrc)
{
    stage_map(B, b, P.stage_cap, S, [&](int t, int src, int w) {
        spos[t] = local_pos<float>(R, S, X, P.nslots, src, w, B.type[src]);
        if (ssrc) ssrc[t] = src;
    });
    if (threadIdx.x == 0) spos[P.stage_cap] = dummy_pos<float4>();
}

// Threshold r^2 < c2 decided on the staged FP32 distance outside a band around c2 that is
// wider than the staging's rounding (its error in r^2 stays below 2e-5 for brick-local
// coordinates), and inside the band by the FP64 expression of the plain definition.
struct Band {
    float lo, hi;
    double c2;
};

__device__ __forceinline__ Band make_band(double c2)
{
    return Band{(float)(c2 * (1.0 - 2e-5) - 1e-4), (float)(c2 * (1.0 + 2e-5) + 1e-4), c2};
}

__device__ __forceinline__ bool within(float r2f, const Band &bd, const RepDev &R, const double *X,
                                       int64_t S_, int64_t i, int64_t j)
{
    if (r2f < bd.lo) return true;
    if (!(r2f < bd.hi)) return false;
    double wi[3];
    for (int a = 0; a < 3; ++a) wi[a] = wrap1(X[3 * i + a], R.L[a]);
    return obs_r2(R, X, S_, wi, j) < bd.c2;
}

__device__ __forceinline__ float staged_r2(const float4 &a, const float4 &b)
{
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return dx * dx + dy * dy + dz * dz;
}

// Observables of valency control: for every own particle the number of list neighbours
// within the attraction range and within the repulsive core of the pair, each threshold
// decided by `within` (exactly as the plain FP64 definition on the wrapped positions), plus
// per-replica sums {sum z, #(z > f), sum p}.  The list holds every pair within the
// interaction cutoff.
__global__ void k_observe(Buffers B, Launch P, int cur, int32_t *__restrict__ z_out,
                          int32_t *__restrict__ pen_out, int64_t *__restrict__ sums)
{
    extern __shared__ __align__(16) float4 spos[];  // [stage_cap + 1]
    __shared__ StageHdr S;
    __shared__ unsigned long long tot[3];
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) {
        pass_header(R, B, b, lb, P.stage_cap, S);
        tot[0] = tot[1] = tot[2] = 0ull;
    }
    __syncthreads();
    if (S.overflow) return;
    const int64_t S_ = P.nslots;
    const double *X = B.x[cur];
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    stage_bonds(B, P, R, S, b, X, spos, nullptr);
    __syncthreads();
    const bool one = R.ntypes == 1;
    const Band ba0 = make_band(R.pair[0].ra2), br0 = make_band(R.pair[0].rr2);
    unsigned long long zs = 0, over = 0, ps = 0;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        const float4 pi = spos[t];
        const int ti = (int)pi.w;
        int z = 0, p = 0;
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            if (R.excl_span > 0) u &= 0x7fff;
            const float4 pj = spos[u];
            const float r2f = staged_r2(pi, pj);
            Band ba = ba0, br = br0;
            if (!one) {
                const PairDev &pd = R.pair[ti * MAXT + (int)pj.w];
                ba = make_band(pd.ra2);
                br = make_band(pd.rr2);
            }
            if (!(r2f < ba.hi) && !(r2f < br.hi)) return;  // beyond both (and the padding)
            z += within(r2f, ba, R, X, S_, i, sm[u]) ? 1 : 0;
            p += within(r2f, br, R, X, S_, i, sm[u]) ? 1 : 0;
        });
        const int32_t tg = B.tag[i];
        if (z_out) z_out[R.o_off + tg] = z;
        if (pen_out) pen_out[R.o_off + tg] = p;
        zs += (unsigned long long)z;
        ps += (unsigned long long)p;
        over += ((double)z > R.pair[ti * MAXT + ti].f) ? 1ull : 0ull;
    }
    zs = wave_sum(zs);
    over = wave_sum(over);
    ps = wave_sum(ps);
    if ((threadIdx.x % VBC_WAVE) == 0) {
        atomicAdd(&tot[0], zs);
        atomicAdd(&tot[1], over);
        atomicAdd(&tot[2], ps);
    }
    __syncthreads();
    if (sums && threadIdx.x < 3 && tot[threadIdx.x])
        atomicAdd((unsigned long long *)&sums[3 * r + threadIdx.x], tot[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// clusters of the bond graph (Section 3): union-find over the slots
// ---------------------------------------------------------------------------
//
// parent[] forms a forest over the slots in which every pointer goes to a smaller slot:
// hooking links a root under a smaller root, and path halving only ever replaces a parent
// by one of its ancestors.  Every walk therefore ends, whatever other lanes do meanwhile,
// and the root of a cluster is its smallest slot.

__device__ __forceinline__ int32_t cc_ld(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void cc_st(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t cc_find(int32_t *parent, int32_t x)
{
    while (true) {
        const int32_t p = cc_ld(parent + x);
        if (p == x) return x;
        const int32_t g = cc_ld(parent + p);
        if (g == p) return p;
        cc_st(parent + x, g);  // path halving
        x = g;
    }
}

__device__ __forceinline__ void cc_union(int32_t *parent, int32_t a, int32_t b)
{
    a = cc_find(parent, a);
    b = cc_find(parent, b);
    while (a != b) {
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(parent + a, a, b);
        if (old == a) return;
        a = cc_find(parent, old);
        b = cc_find(parent, b);
    }
}

__global__ void k_cc_init(ClusterWork W, int64_t S_)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S_; i += (int64_t)gridDim.x * blockDim.x) {
        W.parent[i] = (int32_t)i;
        W.size[i] = 0;
        W.ends[i] = 0u;
        W.mintag[i] = INT32_MAX;
        W.z[i] = 0;
    }
}

// LDS union-find over the own particles of one brick (their staged index is their index in
// the brick), with the same smaller-root rule.
__device__ __forceinline__ int32_t lcc_find(int32_t *lp, int32_t x)
{
    while (true) {
        const int32_t p = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x) return x;
        const int32_t g = __hip_atomic_load(lp + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (g == p) return p;
        __hip_atomic_store(lp + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
    }
}

__device__ __forceinline__ void lcc_union(int32_t *lp, int32_t a, int32_t b)
{
    a = lcc_find(lp, a);
    b = lcc_find(lp, b);
    while (a != b) {
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(lp + a, a, b);
        if (old == a) return;
        a = lcc_find(lp, old);
        b = lcc_find(lp, b);
    }
}

// Bonds of every own particle (the z_i criterion of the observables) from its list.  Bonds
// between two own particles of the brick are joined in LDS first; the forest then starts
// from the brick's local components, each a star under its smallest slot.
__global__ void k_cc_local(Buffers B, Launch P, int cur, ClusterWork W)
{
    extern __shared__ __align__(16) float4 spos[];  // [stage_cap + 1], then lp[bcap]
    __shared__ StageHdr S;
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) pass_header(R, B, b, lb, P.stage_cap, S);
    __syncthreads();
    if (S.overflow) return;
    const int64_t S_ = P.nslots;
    const double *X = B.x[cur];
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    int32_t *lp = (int32_t *)(spos + P.stage_cap + 1);
    stage_bonds(B, P, R, S, b, X, spos, nullptr);
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) lp[t] = t;
    __syncthreads();
    const bool one = R.ntypes == 1;
    const Band ba0 = make_band(R.pair[0].ra2);
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        const float4 pi = spos[t];
        const int ti = (int)pi.w;
        int z = 0;
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            if (R.excl_span > 0) u &= 0x7fff;
            const float4 pj = spos[u];
            const float r2f = staged_r2(pi, pj);
            const Band ba = one ? ba0 : make_band(R.pair[ti * MAXT + (int)pj.w].ra2);
            if (!(r2f < ba.hi)) return;  // also the padding
            if (!within(r2f, ba, R, X, S_, i, sm[u])) return;
            ++z;
            if (u < S.n_own && u > t) lcc_union(lp, t, u);
        });
        W.z[i] = z;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x)
        W.parent[S.base + t] = (int32_t)(S.base + lcc_find(lp, t));
}

// Bonds that leave the brick join the global forest (each once, from its smaller slot).  A
// bond is taken between the current parents of its ends (ancestors, so in the same clusters),
// and a workgroup joins each distinct pair of them once: a condensed brick has hundreds of
// bonds into a few dozen neighbouring components.  The set of pairs lives in LDS with open
// addressing; when it is full the join simply runs.
constexpr int CC_SET = 512;

__global__ void k_cc_hook(Buffers B, Launch P, int cur, ClusterWork W)
{
    extern __shared__ __align__(16) float4 spos[];  // [stage_cap + 1], ssrc[stage_cap], set
    __shared__ StageHdr S;
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) pass_header(R, B, b, lb, P.stage_cap, S);
    __syncthreads();
    if (S.overflow) return;
    const int64_t S_ = P.nslots;
    const double *X = B.x[cur];
    int32_t *ssrc = (int32_t *)(spos + P.stage_cap + 1);
    unsigned long long *set =
        (unsigned long long *)(((uintptr_t)(ssrc + P.stage_cap) + 15) & ~(uintptr_t)15);
    stage_bonds(B, P, R, S, b, X, spos, ssrc);
    for (int k = threadIdx.x; k < CC_SET; k += blockDim.x) set[k] = ~0ull;
    __syncthreads();
    const bool one = R.ntypes == 1;
    const Band ba0 = make_band(R.pair[0].ra2);
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        if (W.z[i] == 0) continue;
        const float4 pi = spos[t];
        const int ti = (int)pi.w;
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            if (R.excl_span > 0) u &= 0x7fff;
            if (u < S.n_own || u == P.stage_cap) return;  // inside the brick, or padding
            const int64_t j = ssrc[u];
            if (j < i) return;
            const float4 pj = spos[u];
            const float r2f = staged_r2(pi, pj);
            const Band ba = one ? ba0 : make_band(R.pair[ti * MAXT + (int)pj.w].ra2);
            if (!(r2f < ba.hi) || !within(r2f, ba, R, X, S_, i, j)) return;
            int32_t pa = cc_ld(W.parent + i), pb = cc_ld(W.parent + j);
            if (pa == pb) return;
            if (pa > pb) {
                const int32_t tmp = pa;
                pa = pb;
                pb = tmp;
            }
            const unsigned long long key = ((unsigned long long)(uint32_t)pa << 32) | (uint32_t)pb;
            unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 55) & (CC_SET - 1);
            for (int probe = 0; probe < 16; ++probe) {
                const unsigned long long prev = atomicCAS(set + h, ~0ull, key);
                if (prev == key) return;  // this pair is joined already
                if (prev == ~0ull) break;  // first of its pair
                h = (h + 1) & (CC_SET - 1);
            }
            cc_union(W.parent, pa, pb);
        });
    }
}

// Size, bond ends and smallest tag of every cluster, gathered at its root; each particle
// keeps its root as parent for the labelling pass.  A workgroup first sums the particles
// of the cluster of its first particle in LDS (in a condensed fluid nearly all of them),
// so that the root of a large cluster takes one atomic per workgroup, not per particle.
__global__ void k_cc_count(Buffers B, Launch P, ClusterWork W)
{
    __shared__ StageHdr S;
    __shared__ int32_t broot, bmin;
    __shared__ uint32_t bsize, bends;
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) {
        pass_header(R, B, b, lb, P.stage_cap, S);
        broot = -1;
        bmin = INT32_MAX;
        bsize = 0u;
        bends = 0u;
    }
    __syncthreads();
    if (S.overflow || S.n_own == 0) return;
    if (threadIdx.x == 0) broot = cc_find(W.parent, (int32_t)S.base);
    __syncthreads();
    const int32_t br = broot;
    uint32_t ls = 0u, le = 0u;
    int32_t lm = INT32_MAX;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        const int32_t root = cc_find(W.parent, (int32_t)i);
        const int32_t tg = B.tag[i];
        if (root == br) {
            ls += 1u;
            le += (uint32_t)W.z[i];
            lm = tg < lm ? tg : lm;
        } else {
            atomicAdd(W.size + root, 1);
            atomicAdd(W.ends + root, (uint32_t)W.z[i]);
            atomicMin(W.mintag + root, tg);
        }
        cc_st(W.parent + i, root);
    }
    ls = wave_sum(ls);
    le = wave_sum(le);
    for (int o = VBC_WAVE / 2; o > 0; o >>= 1) {
        const int32_t v = __shfl_down(lm, o, VBC_WAVE);
        lm = v < lm ? v : lm;
    }
    if ((threadIdx.x % VBC_WAVE) == 0 && ls) {
        atomicAdd(&bsize, ls);
        atomicAdd(&bends, le);
        atomicMin(&bmin, lm);
    }
    __syncthreads();
    if (threadIdx.x == 0 && bsize) {
        atomicAdd(W.size + br, (int32_t)bsize);
        atomicAdd(W.ends + br, bends);
        atomicMin(W.mintag + br, bmin);
    }
}

// Per particle: its cluster's smallest tag.  Per root: the cluster's statistics and its
// histogram bins (all clusters, acyclic clusters).
__global__ void k_cc_label(Buffers B, Launch P, ClusterWork W, int32_t *__restrict__ label,
                           int64_t *__restrict__ stats, int64_t *__restrict__ hist, int hist_len)
{
    __shared__ StageHdr S;
    __shared__ unsigned long long tot[4];
    __shared__ unsigned long long big;
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) {
        pass_header(R, B, b, lb, P.stage_cap, S);
        tot[0] = tot[1] = tot[2] = tot[3] = 0ull;
        big = 0ull;
    }
    __syncthreads();
    if (S.overflow) return;
    unsigned long long nc = 0, cp = 0, bonds = 0, ncyc = 0, lg = 0;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        const int32_t root = W.parent[i];
        if (label) label[R.o_off + B.tag[i]] = W.mintag[root];
        if (root != (int32_t)i) continue;
        const unsigned long long sz = (unsigned long long)W.size[i];
        const unsigned long long e = (unsigned long long)(W.ends[i] / 2u);
        const bool cyc = e >= sz;
        nc += 1ull;
        bonds += e;
        if (cyc) {
            cp += sz;
            ncyc += 1ull;
        }
        lg = sz > lg ? sz : lg;
        if (hist) {
            const int bin = sz < (unsigned long long)hist_len ? (int)sz : 0;
            int64_t *h = hist + (size_t)r * 2 * hist_len;
            atomicAdd((unsigned long long *)(h + bin), 1ull);
            if (!cyc) atomicAdd((unsigned long long *)(h + hist_len + bin), 1ull);
        }
    }
    nc = wave_sum(nc);
    cp = wave_sum(cp);
    bonds = wave_sum(bonds);
    ncyc = wave_sum(ncyc);
    for (int o = VBC_WAVE / 2; o > 0; o >>= 1) {
        const unsigned long long v = __shfl_down(lg, o, VBC_WAVE);
        lg = v > lg ? v : lg;
    }
    if ((threadIdx.x % VBC_WAVE) == 0) {
        atomicAdd(&tot[0], nc);
        atomicAdd(&tot[1], cp);
        atomicAdd(&tot[2], bonds);
        atomicAdd(&tot[3], ncyc);
        atomicMax(&big, lg);
    }
    __syncthreads();
    if (stats && threadIdx.x == 0 && tot[0]) {
        // only workgroups that hold a root have anything to add
        unsigned long long *st = (unsigned long long *)(stats + 5 * (size_t)r);
        atomicAdd(st + 0, tot[0]);
        atomicMax(st + 1, big);
        if (tot[1]) atomicAdd(st + 2, tot[1]);
        if (tot[2]) atomicAdd(st + 3, tot[2]);
        if (tot[3]) atomicAdd(st + 4, tot[3]);
    }
}

// ---------------------------------------------------------------------------
// bond lifetimes (Section 4): partners of every particle carried from sample to sample
// ---------------------------------------------------------------------------

// One sample of the bond tracker.  For every own particle the state (by caller index) holds
// up to M partner tags with the step each bond was first seen (-1: present when tracking
// began).  A stored partner that is no longer bonded is a broken bond: its lifetime goes to
// the replica's histogram (bin = lifetime / bin_steps, the last bin holds the longer ones),
// or to the censored count without a birth.  A bonded particle not stored is a new bond,
// born now.  Each event is counted at the end with the smaller tag, once per bond.
// stats per replica: {formed, broken with a lifetime, broken without one, partners that did
// not fit, bonds now}.
__global__ void k_bond_track(Buffers B, Launch P, int cur, BondTrack T, int reset,
                             int64_t *__restrict__ hist, int hist_len, int64_t bin_steps,
                             int64_t *__restrict__ stats)
{
    extern __shared__ __align__(16) float4 spos[];  // [stage_cap + 1], then stag[stage_cap]
    __shared__ StageHdr S;
    __shared__ unsigned long long tot[5];
    int b, r;
    if (!resolve_brick(P, B, b, r)) return;
    const RepDev &R = B.reps[r];
    const int lb = b - R.b_off;
    if (threadIdx.x == 0) {
        pass_header(R, B, b, lb, P.stage_cap, S);
        for (int k = 0; k < 5; ++k) tot[k] = 0ull;
    }
    __syncthreads();
    if (S.overflow) return;
    const int64_t S_ = P.nslots;
    const double *X = B.x[cur];
    const int32_t *sm = B.smap + (size_t)b * P.stage_cap;
    int32_t *stag = (int32_t *)(spos + P.stage_cap + 1);
    stage_map(B, b, P.stage_cap, S, [&](int t, int src, int w) {
        spos[t] = local_pos<float>(R, S, X, S_, src, w, B.type[src]);
        stag[t] = B.tag[src];
    });
    if (threadIdx.x == 0) spos[P.stage_cap] = dummy_pos<float4>();
    __syncthreads();
    const bool one = R.ntypes == 1;
    const Band ba0 = make_band(R.pair[0].ra2);
    const int M = T.M;
    const int64_t now = (int64_t)B.step[r];
    unsigned long long formed = 0, broken = 0, cens = 0, over = 0, bonds = 0;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        const int64_t i = S.base + t;
        const float4 pi = spos[t];
        const int ti = (int)pi.w;
        const int32_t tg = stag[t];
        const int64_t c = R.o_off + tg;
        int32_t *ptag = T.tags + c * M;
        int64_t *pbirth = T.births + c * M;
        auto bonded = [&](int u) {
            const float4 pj = spos[u];
            const float r2f = staged_r2(pi, pj);
            const Band ba = one ? ba0 : make_band(R.pair[ti * MAXT + (int)pj.w].ra2);
            return r2f < ba.hi && within(r2f, ba, R, X, S_, i, sm[u]);
        };
        int n = 0;
        if (!reset) {
            // 1. which stored partners are still bonded
            const int n_old = min(max(T.count[c], 0), M);
            uint64_t keep = 0ull;
            for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
                if (R.excl_span > 0) u &= 0x7fff;
                if (u == P.stage_cap || !bonded(u)) return;
                const int32_t tj = stag[u];
                for (int k = 0; k < n_old; ++k)
                    if (ptag[k] == tj) {
                        keep |= 1ull << k;
                        break;
                    }
            });
            // 2. broken bonds leave, the others close up in order
            for (int k = 0; k < n_old; ++k) {
                const int32_t tk = ptag[k];
                const int64_t bk = pbirth[k];
                if ((keep >> k) & 1ull) {
                    ptag[n] = tk;
                    pbirth[n] = bk;
                    ++n;
                } else if (tg < tk) {
                    if (bk >= 0) {
                        ++broken;
                        if (hist) {
                            const int64_t bin = (now - bk) / bin_steps;
                            atomicAdd((unsigned long long *)(hist + (size_t)r * hist_len +
                                                             (bin < hist_len - 1 ? bin : hist_len - 1)),
                                      1ull);
                        }
                    } else {
                        ++cens;
                    }
                }
            }
        }
        // 3. bonds not stored are new (at a reset: present from the start, birth unknown)
        const int n_keep = n;
        for_each_neighbour(B.nl, S_, i, B.nn[i], [&](int u) {
            if (R.excl_span > 0) u &= 0x7fff;
            if (u == P.stage_cap || !bonded(u)) return;
            const int32_t tj = stag[u];
            if (tg < tj) ++bonds;
            for (int k = 0; k < n_keep; ++k)
                if (ptag[k] == tj) return;
            if (n < M) {
                ptag[n] = tj;
                pbirth[n] = reset ? (int64_t)-1 : now;
                ++n;
                if (!reset && tg < tj) ++formed;
            } else {
                ++over;
            }
        });
        T.count[c] = n;
    }
    formed = wave_sum(formed);
    broken = wave_sum(broken);
    cens = wave_sum(cens);
    over = wave_sum(over);
    bonds = wave_sum(bonds);
    if ((threadIdx.x % VBC_WAVE) == 0) {
        atomicAdd(&tot[0], formed);
        atomicAdd(&tot[1], broken);
        atomicAdd(&tot[2], cens);
        atomicAdd(&tot[3], over);
        atomicAdd(&tot[4], bonds);
    }
    __syncthreads();
    if (stats && threadIdx.x < 5 && tot[threadIdx.x])
        atomicAdd((unsigned long long *)(stats + 5 * (size_t)r + threadIdx.x), tot[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
static inline unsigned brick_grid(int nb) { return (unsigned)(((nb + 7) / 8) * 8); }

static size_t tabs_bytes(const Launch &P)
{
    int nh_cap = (P.nh_max + 3) & ~3;
    return ((size_t)5 * nh_cap * sizeof(int) + 31) & ~(size_t)31;
}

static size_t sort_bytes(const Launch &P)
{
    return (size_t)4 * P.bcap_max * sizeof(int) + (size_t)3 * P.ncb_max * sizeof(int);
}

size_t lds_bytes_sort(const Launch &P) { return tabs_bytes(P) + sort_bytes(P); }
size_t lds_bytes_nlist(const Launch &P)
{
    // tables, grid-order positions (16 B), cell offsets, grid -> staging order (2 B)
    const size_t nh_cap = (size_t)((P.nh_max + 3) & ~3);
    return tabs_bytes(P) + (size_t)(P.stage_cap + SCAN_UNROLL) * 16 + (nh_cap + 4) * sizeof(int) +
           (size_t)P.stage_cap * 2;
}
size_t lds_bytes_count(const Launch &P)
{
    return (size_t)(P.stage_cap + 1) * (P.precision == VBC_FP64 ? 32 : (P.multi ? 16 : 12));
}
size_t lds_bytes_embed(const Launch &P) { (void)P; return 0; }
// bond tests (observables, clusters): FP32 staging, then the slots or the brick's forest
size_t lds_bytes_bonds(const Launch &P)
{
    return (size_t)(P.stage_cap + 1) * 16 + (size_t)std::max(P.stage_cap, P.bcap_max) * sizeof(int32_t) + 16 +
           CC_SET * sizeof(unsigned long long);
}
size_t lds_bytes_force(const Launch &P)
{
    const size_t real = P.precision == VBC_FP64 ? 8 : 4;
    return (size_t)(P.stage_cap + 1) * real * (P.multi ? 6 : 5);
}

namespace {
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
thread_local int g_ev_used = 0;
thread_local hipError_t g_ev_err = hipSuccess;

// A launch of a timed pass: through hipExtLaunchKernel while timing events are set (its
// error, if any, is kept for launch_events_used's caller), else the plain launch.
template <typename... P, typename... A>
inline void tlaunch(void (*k)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s, A... a)
{
    if (g_ev_stop) {
        std::tuple<std::decay_t<P>...> args(a...);
        void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
        std::apply(
            [&](auto &...x) {
                int n = 0;
                ((ptrs[n++] = (void *)&x), ...);
            },
            args);
        const hipError_t e = hipExtLaunchKernel((const void *)k, grid, block, ptrs, lds, s, g_ev_start,
                                                g_ev_stop, 0);
        if (e != hipSuccess && g_ev_err == hipSuccess) g_ev_err = e;
        g_ev_start = nullptr;
        ++g_ev_used;
    } else {
        k<<<grid, block, lds, s>>>(a...);
    }
}
}  // namespace

void set_launch_events(hipEvent_t start, hipEvent_t stop)
{
    g_ev_start = start;
    g_ev_stop = stop;
    g_ev_used = 0;
    g_ev_err = hipSuccess;
}

int launch_events_used() { return g_ev_used; }

hipError_t launch_events_error() { return g_ev_err; }

hipError_t launch_set_state(const Buffers &B, const Launch &P, int cur, int r, int64_t n,
                            const double *x, const double *v, const int32_t *type,
                            int64_t in_off, int64_t in_stride, uint64_t step0, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_set_state<<<blocks_for(n, 256), 256, 0, s>>>(B, P.nslots, cur, r, in_off, in_stride, x, v,
                                                    type, step0);
    return hipGetLastError();
}

hipError_t launch_get_state(const Buffers &B, const Launch &P, int cur, int r, int64_t nslot,
                            int64_t out_off, int64_t out_stride, double *x, double *v,
                            hipStream_t s)
{
    if (nslot <= 0) return hipSuccess;
    k_get_state<<<blocks_for(nslot, 256), 256, 0, s>>>(B, P.nslots, cur, r, out_off, out_stride,
                                                        x, v);
    return hipGetLastError();
}

hipError_t launch_flags(const Buffers &B, int r_lo, int r_n, uint32_t bits, bool set,
                        hipStream_t s)
{
    if (r_n <= 0) return hipSuccess;
    k_flags<<<blocks_for(r_n, 64), 64, 0, s>>>(B, r_lo, r_n, bits, set ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_admit(const Buffers &B, int r, int64_t nthreads, hipStream_t s)
{
    k_admit<<<blocks_for(std::max<int64_t>(nthreads, 1), 256), 256, 0, s>>>(B, r);
    return hipGetLastError();
}

hipError_t launch_retire(const Buffers &B, int r, int b_off, int nbrick, hipStream_t s)
{
    k_retire<<<blocks_for(std::max(nbrick, 1), 256), 256, 0, s>>>(B, r, b_off, nbrick);
    return hipGetLastError();
}

hipError_t launch_stamp(const Buffers &B, hipStream_t s)
{
    k_stamp<<<1, 1, 0, s>>>(B, (uint32_t)(STAMP_CAP - 1));
    return hipGetLastError();
}

// Full build of replica r (P covering its bricks): bin and sort it from caller-order
// input, then build its list.  k_resort skips FULL replicas, so the same two-kernel tail
// as an incremental rebuild serves.
hipError_t launch_full_build(const Buffers &B, const Launch &P, int cur, int r, int64_t n,
                             hipStream_t s)
{
    if (n > 0) tlaunch(k_gbin, blocks_for(n, 256), 256, 0, s, B, P.nslots, cur, r);
    tlaunch(k_gsort, brick_grid(P.nb_launch), P.block, sort_bytes(P), s, B, P, cur);
    tlaunch(k_nlist, brick_grid(P.nb_launch), P.block, lds_bytes_nlist(P), s, B, P, cur);
    return hipGetLastError();
}

// Incremental rebuild of the replicas whose REBUILD flag is set.  A capacity-wide launch
// first makes the step's work lists and visits only the bricks of those replicas.
hipError_t launch_rebuild(const Buffers &B, const Launch &P, int cur, hipStream_t s)
{
    Launch Q = P;
    if (P.list >= 0) {
        tlaunch(k_worklist, 1, 1024, 0, s, B, P.nrep);
        Q.list = 1;
    }
    tlaunch(k_resort, brick_grid(Q.nb_launch), Q.block, lds_bytes_sort(Q), s, B, Q, cur);
    tlaunch(k_nlist, brick_grid(Q.nb_launch), Q.block, lds_bytes_nlist(Q), s, B, Q, cur);
    return hipGetLastError();
}

template <class Real, bool MULTI>
static void launch_count_t(const Buffers &B, const Launch &P, int cur, double *n_out, int advance,
                           bool stats, hipStream_t s)
{
    size_t lds = lds_bytes_count(P);
    unsigned g = brick_grid(P.nb_launch);
    if (P.one) {
        const OneRep<true> R1{*P.one};
        if (stats) tlaunch(k_count<Real, MULTI, true, true>, g, P.block, lds, s, B, P, cur, n_out, advance, R1);
        else tlaunch(k_count<Real, MULTI, false, true>, g, P.block, lds, s, B, P, cur, n_out, advance, R1);
    } else {
        const OneRep<false> R1{0};
        if (stats) tlaunch(k_count<Real, MULTI, true, false>, g, P.block, lds, s, B, P, cur, n_out, advance, R1);
        else tlaunch(k_count<Real, MULTI, false, false>, g, P.block, lds, s, B, P, cur, n_out, advance, R1);
    }
}

hipError_t launch_count(const Buffers &B, const Launch &P, int cur, double *n_out, int advance,
                        bool stats, hipStream_t s)
{
    bool multi = P.multi != 0;
    if (P.precision == VBC_FP64) {
        if (multi) launch_count_t<double, true>(B, P, cur, n_out, advance, stats, s);
        else launch_count_t<double, false>(B, P, cur, n_out, advance, stats, s);
    } else {
        if (multi) launch_count_t<float, true>(B, P, cur, n_out, advance, stats, s);
        else launch_count_t<float, false>(B, P, cur, n_out, advance, stats, s);
    }
    return hipGetLastError();
}

hipError_t launch_embed(const Buffers &B, const Launch &P, int cur, hipStream_t s)
{
    unsigned g = brick_grid(P.nb_launch);
    bool multi = P.multi != 0;
    const int bs = EMBED_WAVES * VBC_WAVE;
    size_t lds = 0;
    if (P.precision == VBC_FP64) {
        if (multi) tlaunch(k_embed<double, true>, g, bs, lds, s, B, P, cur);
        else tlaunch(k_embed<double, false>, g, bs, lds, s, B, P, cur);
    } else {
        if (multi) tlaunch(k_embed<float, true>, g, bs, lds, s, B, P, cur);
        else tlaunch(k_embed<float, false>, g, bs, lds, s, B, P, cur);
    }
    return hipGetLastError();
}

template <class Real, bool MULTI>
static void launch_force_t(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                           const StepArgs &st, double *F_out, double *e_out, hipStream_t s)
{
    size_t lds = lds_bytes_force(P);
    unsigned g = brick_grid(P.nb_launch);
    if (P.one) {
        const OneRep<true> R1{*P.one};
        if (thermo)
            tlaunch(k_force<Real, MULTI, true, true>, g, P.block, lds, s, B, P, cur, (int)mode, st, F_out, e_out, R1);
        else
            tlaunch(k_force<Real, MULTI, false, true>, g, P.block, lds, s, B, P, cur, (int)mode, st, F_out, e_out, R1);
    } else {
        const OneRep<false> R1{0};
        if (thermo)
            tlaunch(k_force<Real, MULTI, true, false>, g, P.block, lds, s, B, P, cur, (int)mode, st, F_out, e_out, R1);
        else
            tlaunch(k_force<Real, MULTI, false, false>, g, P.block, lds, s, B, P, cur, (int)mode, st, F_out, e_out, R1);
    }
}

hipError_t launch_force(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                        const StepArgs &st, double *F_out, double *e_out, hipStream_t s)
{
    bool multi = P.multi != 0;
    if (P.precision == VBC_FP64) {
        if (multi) launch_force_t<double, true>(B, P, cur, mode, thermo, st, F_out, e_out, s);
        else launch_force_t<double, false>(B, P, cur, mode, thermo, st, F_out, e_out, s);
    } else {
        if (multi) launch_force_t<float, true>(B, P, cur, mode, thermo, st, F_out, e_out, s);
        else launch_force_t<float, false>(B, P, cur, mode, thermo, st, F_out, e_out, s);
    }
    return hipGetLastError();
}

hipError_t launch_thermo_acc(const Buffers &B, const Launch &P, hipStream_t s)
{
    k_thermo_acc<<<P.nrep, 256, 0, s>>>(B, P.nrep);
    return hipGetLastError();
}

hipError_t launch_thermo_clear(const Buffers &B, int nrep, hipStream_t s)
{
    const int n = nrep * THERMO_WORDS;
    k_thermo_clear<<<blocks_for(n, 256), 256, 0, s>>>(B, n);
    return hipGetLastError();
}

hipError_t launch_reduce(const Buffers &B, const Launch &P, double *UW, hipStream_t s)
{
    k_reduce<<<P.nrep, 256, 0, s>>>(B, P.nrep, UW);
    return hipGetLastError();
}

hipError_t launch_kick_drift(const Buffers &B, const Launch &P, int cur, const StepArgs &st,
                             hipStream_t s)
{
    if (P.list >= 0) k_worklist<<<1, 1024, 0, s>>>(B, P.nrep);
    k_kick_drift<<<brick_grid(P.nb_launch), 256, 0, s>>>(B, P, cur, st);
    return hipGetLastError();
}

hipError_t launch_observe(const Buffers &B, const Launch &P, int cur, int32_t *z_out,
                          int32_t *pen_out, int64_t *sums, hipStream_t s)
{
    if (sums) k_zero_i64<<<blocks_for(3 * P.nrep, 256), 256, 0, s>>>(sums, 3 * P.nrep);
    k_observe<<<brick_grid(P.nb_launch), P.block, lds_bytes_bonds(P), s>>>(B, P, cur, z_out, pen_out, sums);
    return hipGetLastError();
}

hipError_t launch_clusters(const Buffers &B, const Launch &P, int cur, const ClusterWork &W,
                           int32_t *label, int64_t *stats, int64_t *hist, int hist_len, hipStream_t s)
{
    if (stats) k_zero_i64<<<blocks_for(5 * P.nrep, 256), 256, 0, s>>>(stats, 5 * P.nrep);
    if (hist) k_zero_i64<<<blocks_for(2 * (int64_t)P.nrep * hist_len, 256), 256, 0, s>>>(hist, 2 * P.nrep * hist_len);
    k_cc_init<<<blocks_for(P.nslots, 256), 256, 0, s>>>(W, P.nslots);
    k_cc_local<<<brick_grid(P.nb_launch), P.block, lds_bytes_bonds(P), s>>>(B, P, cur, W);
    k_cc_hook<<<brick_grid(P.nb_launch), P.block, lds_bytes_bonds(P), s>>>(B, P, cur, W);
    k_cc_count<<<brick_grid(P.nb_launch), P.block, 0, s>>>(B, P, W);
    k_cc_label<<<brick_grid(P.nb_launch), P.block, 0, s>>>(B, P, W, label, stats, hist, hist_len);
    return hipGetLastError();
}

hipError_t launch_bond_track(const Buffers &B, const Launch &P, int cur, const BondTrack &T, int reset,
                             int64_t *hist, int hist_len, int64_t bin_steps, int64_t *stats, hipStream_t s)
{
    if (reset && stats) k_zero_i64<<<blocks_for(5 * P.nrep, 256), 256, 0, s>>>(stats, 5 * P.nrep);
    if (reset && hist) k_zero_i64<<<blocks_for((int64_t)P.nrep * hist_len, 256), 256, 0, s>>>(hist, P.nrep * hist_len);
    k_bond_track<<<brick_grid(P.nb_launch), P.block, lds_bytes_bonds(P), s>>>(B, P, cur, T, reset, hist, hist_len,
                                                                              bin_steps, stats);
    return hipGetLastError();
}

hipError_t launch_export_nlist(const Buffers &B, const Launch &P, int rep, int nbrick,
                               int32_t *pairs, int64_t cap, int64_t *count, hipStream_t s)
{
    unsigned long long *c = (unsigned long long *)count;
    k_zero_u64<<<1, 1, 0, s>>>(c);
    if (nbrick > 0)
        k_export_nlist<<<nbrick, P.block, 0, s>>>(B, P, rep, pairs, cap, c);
    return hipGetLastError();
}

}  // namespace vbc
