// vbc_kernels.hip -- gfx950 kernels of the VBC hot path.
//
// Passes (Section 2, "two passes over the neighbour list"; the force itself follows from
// differentiating eq. (Vhat)):
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
// Data flow of one workgroup: it owns one cell brick; it stages its own particles and the
// one-cell halo around the brick into LDS in a brick-local frame, then sweeps each own
// particle's list (16-bit indices into that staging order) reading neighbours from LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "vbc_internal.h"

namespace vbc {

#define VBC_WAVE 64

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <class T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };
template <class T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

__device__ __forceinline__ float rsqrt_r(float x) { return __frsqrt_rn(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ int rep_of_particle(const RepDev *R, int nrep, int64_t i)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (R[mid].p_off <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int rep_of_brick(const RepDev *R, int nrep, int b)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (R[mid].b_off <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int rep_of_cell(const RepDev *R, int nrep, int c)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (R[mid].c_off <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Map workgroups to bricks so that consecutive bricks (which share halo cells) land on
// the same XCD: workgroups are dealt round-robin over the 8 XCDs, so workgroup g runs on
// XCD g % 8; give that XCD a contiguous run of bricks.  The grid is padded to a multiple
// of 8 and the map is a bijection on [0, grid).
__device__ __forceinline__ int brick_of_block()
{
    int G = gridDim.x;
    int g = blockIdx.x;
    return (g & 7) * (G >> 3) + (g >> 3);
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

template <class Real>
__device__ __forceinline__ Real omega_dr(Real x, Real x1, Real x2)
{
    Real w = x2 - x1;
    Real u = (x - x1) / w;
    if (!(u > Real(0) && u < Real(1))) return Real(0);
    return Real(-4) * u * (Real(1) - u * u) / w;
}

// Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11): two 64x64->128-bit
// multiplies by fixed odd constants per round, high halves xor-ed with the other two
// counter words and the round key; the key is bumped by two Weyl constants per round.
__device__ __forceinline__ void philox4x64_10(uint64_t &c0, uint64_t &c1, uint64_t &c2,
                                              uint64_t &c3, uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// Zero-mean unit-variance uniform variates sqrt(3)(2u - 1) from the first three words,
// u = (word >> 11) 2^-53: only exactly rounded operations.
__device__ __forceinline__ void langevin_noise(uint64_t seed, uint64_t tag, uint64_t step,
                                               double xi[3])
{
#pragma clang fp contract(off)
    uint64_t c0 = step, c1 = 0, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, tag);
    const double SQRT3 = 1.7320508075688772;
    xi[0] = (2.0 * ((double)(c0 >> 11) * 0x1.0p-53) - 1.0) * SQRT3;
    xi[1] = (2.0 * ((double)(c1 >> 11) * 0x1.0p-53) - 1.0) * SQRT3;
    xi[2] = (2.0 * ((double)(c2 >> 11) * 0x1.0p-53) - 1.0) * SQRT3;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = VBC_WAVE / 2; o > 0; o >>= 1) v += __shfl_down(v, o, VBC_WAVE);
    return v;
}

// ---------------------------------------------------------------------------
// state in / out
// ---------------------------------------------------------------------------

__global__ void k_set_state(Buffers B, int nrep, int64_t ntot, int rep_lo, int rep_hi,
                            int64_t in_off, int64_t in_stride, const double *__restrict__ x,
                            const double *__restrict__ v, const int32_t *__restrict__ type,
                            uint64_t step0)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t lo = B.reps[rep_lo].p_off;
    int64_t hi = B.reps[rep_hi].p_off + B.reps[rep_hi].n;
    int64_t k = lo + i;  // internal index == caller index when freshly set
    if (k >= hi) return;
    int r = rep_of_particle(B.reps, nrep, k);
    const RepDev &R = B.reps[r];
    int64_t tg = k - R.p_off;
    int64_t src = R.o_off + tg - in_off;
    for (int a = 0; a < 3; ++a) {
        B.x[0][a * ntot + k] = x[a * in_stride + src];
        B.x[1][a * ntot + k] = x[a * in_stride + src];
        B.v[a * ntot + k] = v ? v[a * in_stride + src] : 0.0;
    }
    B.tag[k] = (int32_t)tg;
    int ty = type ? type[src] : 0;
    B.type[k] = (ty >= 0 && ty < R.ntypes) ? ty : 0;
    B.inv[k] = k;
    if (tg == 0) {
        B.step[r] = step0;
        B.flags[r] = VBC_FLAG_REBUILD;
    }
}

__global__ void k_get_state(Buffers B, int nrep, int64_t ntot, int cur, int rep_lo, int rep_hi,
                            int64_t out_off, int64_t out_stride, double *__restrict__ x,
                            double *__restrict__ v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t lo = B.reps[rep_lo].p_off;
    int64_t hi = B.reps[rep_hi].p_off + B.reps[rep_hi].n;
    int64_t k = lo + i;
    if (k >= hi) return;
    int r = rep_of_particle(B.reps, nrep, k);
    const RepDev &R = B.reps[r];
    int64_t dst = R.o_off + B.tag[k] - out_off;
    for (int a = 0; a < 3; ++a) {
        if (x) {
            double t = B.x[cur][a * ntot + k];
            double L = R.L[a];
            t = t - L * floor(t / L);
            if (t >= L) t -= L;
            if (t < 0.0) t = 0.0;
            x[a * out_stride + dst] = t;
        }
        if (v) v[a * out_stride + dst] = B.v[a * ntot + k];
    }
}

__global__ void k_flags_or(Buffers B, int nrep, uint32_t bits)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrep) B.flags[r] |= bits;
}

__global__ void k_flags_clear(Buffers B, int nrep, uint32_t bits)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrep) B.flags[r] &= ~bits;
}

__global__ void k_advance(Buffers B, int nrep, uint64_t nsteps)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrep) B.step[r] += nsteps;
}

// ---------------------------------------------------------------------------
// neighbour-list build: bin, scan, scatter, sort within cells, list
// ---------------------------------------------------------------------------

// Wrap into the box, bin by cell (edge h >= list radius), count per cell.
__global__ void k_bin(Buffers B, int nrep, int64_t ntot, int cur)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    int r = rep_of_particle(B.reps, nrep, i);
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & VBC_FLAG_REBUILD)) return;
    int c[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
        double t = B.x[cur][a * ntot + i];
        if (!isfinite(t)) {
            bad = true;
            t = 0.0;
        }
        double L = R.L[a];
        if (t < 0.0 || t >= L) {
            t = t - L * floor(t / L);
            if (t >= L) t -= L;
            if (t < 0.0) t = 0.0;
        }
        B.x[cur][a * ntot + i] = t;
        int ca = (int)floor(t / R.h[a]);
        c[a] = ca < 0 ? 0 : (ca >= R.nc[a] ? R.nc[a] - 1 : ca);
    }
    if (bad) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NONFINITE);
    int lin = c[0] + R.nc[0] * (c[1] + R.nc[1] * c[2]);
    int rank = B.cell_rank[R.c_off + lin];
    B.pcs[i] = rank;
    B.slot[i] = atomicAdd(&B.cell_cnt[R.c_off + rank], 1);
}

// Exclusive scan of the cell counts of one replica (one workgroup per replica); the
// counters are cleared for the next build.
__global__ void k_scan(Buffers B, int nrep)
{
    int r = blockIdx.x;
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & VBC_FLAG_REBUILD)) return;
    __shared__ int64_t part[1024];
    int nt = blockDim.x;
    int n = R.ncell;
    int chunk = (n + nt - 1) / nt;
    int lo = threadIdx.x * chunk;
    int hi = min(n, lo + chunk);
    int64_t s = 0;
    for (int k = lo; k < hi; ++k) s += B.cell_cnt[R.c_off + k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int t = 0; t < nt; ++t) {
            int64_t v = part[t];
            part[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int64_t acc = R.p_off + part[threadIdx.x];
    for (int k = lo; k < hi; ++k) {
        int c = B.cell_cnt[R.c_off + k];
        B.cell_start[R.cs_off + k] = acc;
        acc += c;
        B.cell_cnt[R.c_off + k] = 0;
    }
    if (threadIdx.x == 0) B.cell_start[R.cs_off + n] = R.p_off + R.n;
}

__global__ void k_scatter(Buffers B, int nrep, int64_t ntot)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    int r = rep_of_particle(B.reps, nrep, i);
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & VBC_FLAG_REBUILD)) return;
    int64_t dst = B.cell_start[R.cs_off + B.pcs[i]] + B.slot[i];
    B.perm[dst] = (int32_t)i;
}

// One thread per cell: order the cell's particles by tag (so the sorted order depends only
// on positions and tags), then gather every per-particle array into the new order.
__global__ void k_cellsort(Buffers B, int nrep, int64_t ntot, int ncell_tot, int cur)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell_tot) return;
    int r = rep_of_cell(B.reps, nrep, c);
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & VBC_FLAG_REBUILD)) return;
    int rank = c - R.c_off;
    int64_t s = B.cell_start[R.cs_off + rank];
    int64_t e = B.cell_start[R.cs_off + rank + 1];
    for (int64_t p = s + 1; p < e; ++p) {
        int32_t o = B.perm[p];
        int32_t key = B.tag[o];
        int64_t q = p - 1;
        while (q >= s) {
            int32_t oq = B.perm[q];
            if (B.tag[oq] <= key) break;
            B.perm[q + 1] = oq;
            --q;
        }
        B.perm[q + 1] = o;
    }
    for (int64_t p = s; p < e; ++p) {
        int32_t o = B.perm[p];
        for (int a = 0; a < 3; ++a) {
            B.xs[a * ntot + p] = B.x[cur][a * ntot + o];
            B.vs[a * ntot + p] = B.v[a * ntot + o];
        }
        int32_t tg = B.tag[o];
        B.tags[p] = tg;
        B.types[p] = B.type[o];
        B.pcell[p] = rank;
        B.inv[R.p_off + tg] = p;
    }
}

// ---------------------------------------------------------------------------
// brick staging
// ---------------------------------------------------------------------------

struct StageHdr {
    int64_t own_start;
    int n_own;
    int total;
    int rank0;
    int nh;
    int c0[3], e[3], H[3];
    double O[3];
    int overflow;
};

struct StageTabs {
    int *q_off;    // staged offset of each halo-grid cell (own and halo)
    int *q_cnt;    // particles in the cell
    int *q_src;    // first internal index of the cell
    int *q_hpre;   // exclusive prefix of halo-cell counts (own cells contribute 0)
    int *q_w;      // packed image shift (wx+1) | (wy+1) << 2 | (wz+1) << 4
};

__device__ __forceinline__ int unpack_w(int w, int a) { return ((w >> (2 * a)) & 3) - 1; }

// Lay out the staging of brick lb of replica R: the own cells first (one contiguous run
// of the sorted order), then every halo cell of the (e+2)^3 grid in x-fastest order.
// All threads of the block call this.  Uses cell_start of the last build.
__device__ void stage_tables(const RepDev &R, int lb, const Buffers &B, StageHdr &S,
                             StageTabs T, int stage_cap)
{
    if (threadIdx.x == 0) {
        int bx = lb % R.nb[0];
        int by = (lb / R.nb[0]) % R.nb[1];
        int bz = lb / (R.nb[0] * R.nb[1]);
        int Bc[3] = {bx, by, bz};
        int ncb = 1;
        for (int a = 0; a < 3; ++a) {
            S.c0[a] = Bc[a] * R.bd[a];
            S.e[a] = min(R.bd[a], R.nc[a] - S.c0[a]);
            S.H[a] = S.e[a] + 2;
            ncb *= S.e[a];
            S.O[a] = ((double)S.c0[a] + 0.5 * (double)S.e[a]) * R.h[a];
        }
        S.nh = S.H[0] * S.H[1] * S.H[2];
        S.rank0 = B.brick_rank0[R.b_off + lb];
        S.own_start = B.cell_start[R.cs_off + S.rank0];
        S.n_own = (int)(B.cell_start[R.cs_off + S.rank0 + ncb] - S.own_start);
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
        int rank = B.cell_rank[R.c_off + g[0] + R.nc[0] * (g[1] + R.nc[1] * g[2])];
        int64_t st = B.cell_start[R.cs_off + rank];
        int cnt = (int)(B.cell_start[R.cs_off + rank + 1] - st);
        T.q_src[q] = (int)st;
        T.q_cnt[q] = cnt;
        T.q_w[q] = w;
        T.q_off[q] = own ? (int)(st - S.own_start) : -1;
        T.q_hpre[q] = own ? 0 : cnt;
    }
    __syncthreads();
    // exclusive scan of the halo counts by the first wave
    if (threadIdx.x < VBC_WAVE) {
        int lane = threadIdx.x;
        int carry = 0;
        for (int base = 0; base < S.nh; base += VBC_WAVE) {
            int q = base + lane;
            int v = q < S.nh ? T.q_hpre[q] : 0;
            int incl = v;
#pragma unroll
            for (int o = 1; o < VBC_WAVE; o <<= 1) {
                int t = __shfl_up(incl, o, VBC_WAVE);
                if (lane >= o) incl += t;
            }
            if (q < S.nh) T.q_hpre[q] = carry + incl - v;
            carry += __shfl(incl, VBC_WAVE - 1, VBC_WAVE);
        }
        if (lane == 0) {
            S.total = S.n_own + carry;
            S.overflow = S.total > stage_cap;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < S.nh; q += blockDim.x)
        if (T.q_off[q] < 0) T.q_off[q] = S.n_own + T.q_hpre[q];
    __syncthreads();
}

// Internal index and image shift of staged slot t.
__device__ __forceinline__ void stage_source(const StageHdr &S, const StageTabs &T, int t,
                                             int64_t &src, int &w)
{
    if (t < S.n_own) {
        src = S.own_start + t;
        w = 0x15;
        return;
    }
    int k = t - S.n_own;
    int lo = 0, hi = S.nh;  // first q with q_hpre[q] > k
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (T.q_hpre[mid] <= k) lo = mid + 1; else hi = mid;
    }
    int q = lo - 1;
    src = T.q_src[q] + (k - T.q_hpre[q]);
    w = T.q_w[q];
}

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

// List build for one brick: copy the brick's particles from the sorted scratch into the
// live arrays, stage raw FP64 positions of own and halo particles, and list for each own
// particle every staged j != i with minimum-image r^2 < r_list^2.  The distance is the same
// expression as the plain definition -- t = x_i - x_j, d = t - L k with k the image of the
// halo cell, r^2 = (dx dx + dy dy) + dz dz -- without contraction, so the set is exact.
__global__ void k_nlist(Buffers B, Launch P, int cur)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    int b = brick_of_block();
    if (b >= P.nbrick_tot) return;
    int r = rep_of_brick(B.reps, P.nrep, b);
    const RepDev &R = B.reps[r];
    if (!(B.flags[r] & VBC_FLAG_REBUILD)) return;
    int lb = b - R.b_off;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    double *sx = (double *)after_tabs(smem, nh_cap);
    double *sy = sx + P.stage_cap;
    double *sz = sy + P.stage_cap;
    const int64_t ntot = P.ntot;

    stage_tables(R, lb, B, S, T, P.stage_cap);

    // sorted scratch -> live arrays for the own range
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        for (int a = 0; a < 3; ++a) {
            double xa = B.xs[a * ntot + i];
            B.x[cur][a * ntot + i] = xa;
            B.xref[a * ntot + i] = xa;
            B.v[a * ntot + i] = B.vs[a * ntot + i];
        }
        B.tag[i] = B.tags[i];
        B.type[i] = B.types[i];
    }
    if (S.overflow) {
        for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) B.nn[S.own_start + t] = 0;
        if (threadIdx.x == 0) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
        return;
    }
    for (int t = threadIdx.x; t < S.total; t += blockDim.x) {
        int64_t src;
        int w;
        stage_source(S, T, t, src, w);
        sx[t] = B.xs[src];
        sy[t] = B.xs[ntot + src];
        sz[t] = B.xs[2 * ntot + src];
    }
    __syncthreads();

    const double rl2 = R.rlist2;
    bool ovf = false;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        int loc = B.pcell[i] - S.rank0;
        int lx = loc % S.e[0], ly = (loc / S.e[0]) % S.e[1], lz = loc / (S.e[0] * S.e[1]);
        double xi = sx[t], yi = sy[t], zi = sz[t];
        int nn = 0;
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy)
                for (int dx = 0; dx < 3; ++dx) {
                    int q = (lx + dx) + S.H[0] * ((ly + dy) + S.H[1] * (lz + dz));
                    int off = T.q_off[q], cnt = T.q_cnt[q], w = T.q_w[q];
                    double kx = (double)unpack_w(w, 0), ky = (double)unpack_w(w, 1),
                           kz = (double)unpack_w(w, 2);
                    for (int u = off; u < off + cnt; ++u) {
                        if (u == t) continue;
                        double r2;
                        {
#pragma clang fp contract(off)
                            double tx = xi - sx[u], ty = yi - sy[u], tz = zi - sz[u];
                            double ddx = tx - R.L[0] * kx;
                            double ddy = ty - R.L[1] * ky;
                            double ddz = tz - R.L[2] * kz;
                            r2 = (ddx * ddx + ddy * ddy) + ddz * ddz;
                        }
                        if (r2 < rl2) {
                            if (nn < P.k_max) B.nl[(size_t)nn * ntot + i] = (uint16_t)u;
                            ++nn;
                        }
                    }
                }
        if (nn > P.k_max) {
            ovf = true;
            nn = P.k_max;
        }
        B.nn[i] = (uint16_t)nn;
    }
    if (ovf) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NLIST_OVERFLOW);
}

// ---------------------------------------------------------------------------
// pass 1: counts
// ---------------------------------------------------------------------------

// Pair constants converted to the pair-arithmetic precision.
template <class Real>
struct PairR {
    Real E_r, c_r, inv_rr2, E_a, c_a, m, inv_w, r_l, inv_dw, c_c, rl2, rh2, rc2;
    Real x1, x2;
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
    q.attract = p.attract;
    return q;
}

template <class Real>
__device__ __forceinline__ void stage_positions(const RepDev &R, const StageHdr &S,
                                                const StageTabs &T, const double *__restrict__ X,
                                                int64_t ntot, int t, int64_t &src,
                                                typename V4<Real>::t *spos, const int32_t *type)
{
    int w;
    stage_source(S, T, t, src, w);
    typename V4<Real>::t p;
    double lx = (X[src] + R.L[0] * (double)unpack_w(w, 0)) - S.O[0];
    double ly = (X[ntot + src] + R.L[1] * (double)unpack_w(w, 1)) - S.O[1];
    double lz = (X[2 * ntot + src] + R.L[2] * (double)unpack_w(w, 2)) - S.O[2];
    p.x = (Real)lx;
    p.y = (Real)ly;
    p.z = (Real)lz;
    p.w = (Real)type[src];
    spos[t] = p;
}

template <class Real, bool MULTI>
__global__ void k_count(Buffers B, Launch P, int cur, double *__restrict__ n_out)
{
    using R4 = typename V4<Real>::t;
    using R2 = typename V2<Real>::t;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    __shared__ int any_win;
    __shared__ PairR<Real> pt[MAXT * MAXT];
    int b = brick_of_block();
    if (b >= P.nbrick_tot) return;
    int r = rep_of_brick(B.reps, P.nrep, b);
    const RepDev &R = B.reps[r];
    int lb = b - R.b_off;
    if (lb == 0 && threadIdx.x == 0) atomicAnd(&B.flags[r], ~(uint32_t)VBC_FLAG_REBUILD);
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    R4 *spos = (R4 *)after_tabs(smem, nh_cap);
    const int64_t ntot = P.ntot;
    const int nt = R.ntypes;
    if (threadIdx.x < nt * nt) {
        int a = threadIdx.x / nt, c = threadIdx.x % nt;
        pt[a * MAXT + c] = pair_r<Real>(R.pair[a * MAXT + c], R.rc2);
    }
    if (threadIdx.x == 0) any_win = 0;
    stage_tables(R, lb, B, S, T, P.stage_cap);
    R2 *sA = (R2 *)B.sA;
    if (S.overflow) {
        for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
            int64_t i = S.own_start + t;
            B.nd[i] = 0.0;
            sA[i] = R2{Real(0), Real(0)};
        }
        if (threadIdx.x == 0) {
            atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
            B.win[b] = 0;
        }
        return;
    }
    for (int t = threadIdx.x; t < S.total; t += blockDim.x) {
        int64_t src;
        stage_positions<Real>(R, S, T, B.x[cur], ntot, t, src, spos, B.type);
    }
    __syncthreads();

    const PairR<Real> p0 = pt[0];
    bool win = false;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        R4 pi = spos[t];
        int ti = MULTI ? (int)pi.w : 0;
        int nn = B.nn[i];
        const uint16_t *lp = B.nl + i;
        int whole = 0;
        double frac = 0.0;
        for (int s = 0; s < nn; ++s) {
            int u = lp[(size_t)s * ntot];
            R4 pj = spos[u];
            Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            Real r2 = dx * dx + dy * dy + dz * dz;
            if (MULTI) {
                int tj = (int)pj.w;
                if (!((R.mask[ti] >> tj) & 1u)) continue;
                const PairR<Real> &q = pt[ti * MAXT + tj];
                if (r2 <= q.rl2) {
                    ++whole;
                } else if (r2 < q.rh2) {
                    Real rr = sqrt(r2);
                    Real uu = (rr - q.r_l) * q.inv_dw;
                    Real qq = Real(1) - uu * uu;
                    frac += (double)(qq * qq);
                }
            } else {
                if (r2 <= p0.rl2) {
                    ++whole;
                } else if (r2 < p0.rh2) {
                    Real rr = sqrt(r2);
                    Real uu = (rr - p0.r_l) * p0.inv_dw;
                    Real qq = Real(1) - uu * uu;
                    frac += (double)(qq * qq);
                }
            }
        }
        double n = (double)whole + frac;
        B.nd[i] = n;
        if (MULTI) {
            // the switching factor depends on the pair: keep the count itself
            sA[i] = R2{(Real)n, Real(0)};
            for (int u = 0; u < nt; ++u) {
                const PairDev &pd = R.pair[ti * MAXT + u];
                if (pd.attract && n > pd.x1 && n < pd.x2) win = true;
            }
        } else {
            const PairDev &pd = R.pair[0];
            double s = omega_d64(n, pd.x1, pd.x2);
            sA[i] = R2{(Real)s, Real(0)};
            if (pd.attract && n > pd.x1 && n < pd.x2) win = true;
        }
        if (n_out) n_out[R.o_off + B.tag[i]] = n;
    }
    if (win) any_win = 1;
    __syncthreads();
    if (threadIdx.x == 0) B.win[b] = (uint8_t)any_win;
}

// ---------------------------------------------------------------------------
// pass 2a: dU/dn for particles inside a switching window
// ---------------------------------------------------------------------------

template <class Real, bool MULTI>
__global__ void k_embed(Buffers B, Launch P, int cur)
{
    using R4 = typename V4<Real>::t;
    using R2 = typename V2<Real>::t;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    __shared__ PairR<Real> pt[MAXT * MAXT];
    int b = brick_of_block();
    if (b >= P.nbrick_tot) return;
    if (!B.win[b]) return;
    int r = rep_of_brick(B.reps, P.nrep, b);
    const RepDev &R = B.reps[r];
    int lb = b - R.b_off;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    R4 *spos = (R4 *)after_tabs(smem, nh_cap);
    Real *ss = (Real *)(spos + P.stage_cap);
    const int64_t ntot = P.ntot;
    const int nt = R.ntypes;
    if (threadIdx.x < nt * nt) {
        int a = threadIdx.x / nt, c = threadIdx.x % nt;
        pt[a * MAXT + c] = pair_r<Real>(R.pair[a * MAXT + c], R.rc2);
    }
    stage_tables(R, lb, B, S, T, P.stage_cap);
    if (S.overflow) return;
    R2 *sA = (R2 *)B.sA;
    for (int t = threadIdx.x; t < S.total; t += blockDim.x) {
        int64_t src;
        stage_positions<Real>(R, S, T, B.x[cur], ntot, t, src, spos, B.type);
        ss[t] = sA[src].x;
    }
    __syncthreads();
    const PairR<Real> p0 = pt[0];
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        double n_i = B.nd[i];
        R4 pi = spos[t];
        int ti = MULTI ? (int)pi.w : 0;
        double sd_i = 0.0;
        bool any = false;
        if (MULTI) {
            for (int u = 0; u < nt; ++u) {
                const PairDev &pd = R.pair[ti * MAXT + u];
                if (pd.attract && n_i > pd.x1 && n_i < pd.x2) any = true;
            }
        } else {
            sd_i = omega_dd64(n_i, R.pair[0].x1, R.pair[0].x2);
            any = R.pair[0].attract && sd_i != 0.0;
        }
        if (!any) continue;
        int nn = B.nn[i];
        const uint16_t *lp = B.nl + i;
        double acc = 0.0;
        for (int s = 0; s < nn; ++s) {
            int u = lp[(size_t)s * ntot];
            R4 pj = spos[u];
            Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            Real r2 = dx * dx + dy * dy + dz * dz;
            if (MULTI) {
                int tj = (int)pj.w;
                const PairR<Real> &q = pt[ti * MAXT + tj];
                if (!q.attract) continue;
                Real rr = sqrt(r2);
                Real uu = (rr - q.m) * q.inv_w;
                Real qq = Real(1) - uu * uu;
                if (!(qq > Real(0))) continue;
                Real va = -q.E_a * qq * qq;
                const PairDev &pd = R.pair[ti * MAXT + tj];
                double sdi = omega_dd64(n_i, pd.x1, pd.x2);
                if (sdi == 0.0) continue;
                Real sj = omega_r<Real>(ss[u], q.x1, q.x2);
                acc += sdi * (double)(sj * va);
            } else {
                Real rr = sqrt(r2);
                Real uu = (rr - p0.m) * p0.inv_w;
                Real qq = Real(1) - uu * uu;
                if (!(qq > Real(0))) continue;
                acc += (double)(ss[u] * (-p0.E_a * qq * qq));
            }
        }
        double A = MULTI ? acc : sd_i * acc;
        sA[i].y = (Real)A;
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

template <class Real, bool MULTI, bool THERMO>
__global__ void k_force(Buffers B, Launch P, int cur, int mode, StepArgs st,
                        double *__restrict__ F_out, double *__restrict__ e_out)
{
    using R4 = typename V4<Real>::t;
    using R2 = typename V2<Real>::t;
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    __shared__ PairR<Real> pt[MAXT * MAXT];
    __shared__ double red[8][1024 / VBC_WAVE];
    __shared__ int moved;
    int b = brick_of_block();
    if (b >= P.nbrick_tot) return;
    int r = rep_of_brick(B.reps, P.nrep, b);
    const RepDev &R = B.reps[r];
    int lb = b - R.b_off;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    R4 *spos = (R4 *)after_tabs(smem, nh_cap);
    R2 *ssa = (R2 *)(spos + P.stage_cap);
    const int64_t ntot = P.ntot;
    const int nt = R.ntypes;
    if (threadIdx.x < nt * nt) {
        int a = threadIdx.x / nt, c = threadIdx.x % nt;
        pt[a * MAXT + c] = pair_r<Real>(R.pair[a * MAXT + c], R.rc2);
    }
    if (threadIdx.x == 0) moved = 0;
    stage_tables(R, lb, B, S, T, P.stage_cap);
    const R2 *sA = (const R2 *)B.sA;
    if (S.overflow) {
        if (threadIdx.x == 0) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_STAGE_OVERFLOW);
        if (THERMO && threadIdx.x < 8) B.part[(size_t)b * 8 + threadIdx.x] = 0.0;
        return;
    }
    for (int t = threadIdx.x; t < S.total; t += blockDim.x) {
        int64_t src;
        stage_positions<Real>(R, S, T, B.x[cur], ntot, t, src, spos, B.type);
        ssa[t] = sA[src];
    }
    __syncthreads();

    const PairR<Real> p0 = pt[0];
    const uint64_t step = B.step[r] + st.step_off;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // e, W, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz
    bool bad = false, mv = false;
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        R4 pi = spos[t];
        R2 sai = ssa[t];
        int ti = MULTI ? (int)pi.w : 0;
        int nn = B.nn[i];
        const uint16_t *lp = B.nl + i;
        Real fx = 0, fy = 0, fz = 0, ei = 0;
        Real w0 = 0, wxx = 0, wyy = 0, wzz = 0, wxy = 0, wxz = 0, wyz = 0;
        for (int s = 0; s < nn; ++s) {
            int u = lp[(size_t)s * ntot];
            R4 pj = spos[u];
            Real dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
            Real r2 = dx * dx + dy * dy + dz * dz;
            Real phr, ep;
            if (MULTI) {
                int tj = (int)pj.w;
                const PairR<Real> &q = pt[ti * MAXT + tj];
                if (!(r2 < q.rc2)) continue;
                R2 saj = ssa[u];
                Real rinv = rsqrt_r(r2 > Real(1e-30) ? r2 : Real(1e-30));
                Real rr = r2 * rinv;
                Real tc = Real(1) - r2 * q.inv_rr2;
                tc = tc > Real(0) ? tc : Real(0);
                phr = q.c_r * tc;
                ep = q.E_r * tc * tc;
                if (q.attract) {
                    Real uu = (rr - q.m) * q.inv_w;
                    Real qq = Real(1) - uu * uu;
                    if (qq > Real(0)) {
                        Real psi = omega_r<Real>(sai.x, q.x1, q.x2) * omega_r<Real>(saj.x, q.x1, q.x2);
                        ep -= q.E_a * psi * qq * qq;
                        phr += psi * q.c_a * uu * qq * rinv;
                    }
                }
                Real asum = (((R.mask[ti] >> tj) & 1u) ? sai.y : Real(0)) +
                            (((R.mask[tj] >> ti) & 1u) ? saj.y : Real(0));
                Real uc = (rr - q.r_l) * q.inv_dw;
                uc = uc < Real(0) ? Real(0) : (uc > Real(1) ? Real(1) : uc);
                phr += asum * q.c_c * uc * (Real(1) - uc * uc) * rinv;
            } else {
                if (!(r2 < p0.rc2)) continue;
                R2 saj = ssa[u];
                Real rinv = rsqrt_r(r2 > Real(1e-30) ? r2 : Real(1e-30));
                Real rr = r2 * rinv;
                Real tc = Real(1) - r2 * p0.inv_rr2;
                tc = tc > Real(0) ? tc : Real(0);
                phr = p0.c_r * tc;
                ep = p0.E_r * tc * tc;
                Real uu = (rr - p0.m) * p0.inv_w;
                Real qq = Real(1) - uu * uu;
                qq = qq > Real(0) ? qq : Real(0);
                Real psi = sai.x * saj.x;
                ep -= p0.E_a * psi * qq * qq;
                phr += psi * p0.c_a * uu * qq * rinv;
                Real uc = (rr - p0.r_l) * p0.inv_dw;
                uc = uc < Real(0) ? Real(0) : (uc > Real(1) ? Real(1) : uc);
                phr += (sai.y + saj.y) * p0.c_c * uc * (Real(1) - uc * uc) * rinv;
            }
            fx -= phr * dx;
            fy -= phr * dy;
            fz -= phr * dz;
            if (THERMO) {
                ei += ep;
                w0 -= phr * r2;
                wxx -= phr * dx * dx;
                wyy -= phr * dy * dy;
                wzz -= phr * dz * dz;
                wxy -= phr * dx * dy;
                wxz -= phr * dx * dz;
                wyz -= phr * dy * dz;
            }
        }
        double F[3] = {(double)fx, (double)fy, (double)fz};
        double eb = 0.0, wb[7] = {0, 0, 0, 0, 0, 0, 0};
        const double *X = B.x[cur];
        double xi_[3] = {X[i], X[ntot + i], X[2 * ntot + i]};
        int32_t tg = B.tag[i];
        if (R.chain_len > 1) {
            // harmonic bonds to the neighbouring beads of the same chain
            int bead = tg % R.chain_len;
            for (int side = -1; side <= 1; side += 2) {
                if ((side < 0 && bead == 0) || (side > 0 && bead == R.chain_len - 1)) continue;
                int64_t j = B.inv[R.p_off + tg + side];
                double d[3];
                for (int a = 0; a < 3; ++a) {
                    double tt = xi_[a] - X[a * ntot + j];
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
            double e_i = 0.5 * (double)ei + eb;
            acc[0] += e_i;
            acc[1] += 0.5 * (double)w0 + wb[0];
            acc[2] += 0.5 * (double)wxx + wb[1];
            acc[3] += 0.5 * (double)wyy + wb[2];
            acc[4] += 0.5 * (double)wzz + wb[3];
            acc[5] += 0.5 * (double)wxy + wb[4];
            acc[6] += 0.5 * (double)wxz + wb[5];
            acc[7] += 0.5 * (double)wyz + wb[6];
            if (e_out) e_out[R.o_off + tg] = e_i;
        }
        if (mode == MODE_EVAL) {
            for (int a = 0; a < 3; ++a) B.Fst[a * ntot + i] = F[a];
            if (F_out)
                for (int a = 0; a < 3; ++a) F_out[a * ntot + R.o_off + tg] = F[a];
        } else {
            double vv[3] = {B.v[i], B.v[ntot + i], B.v[2 * ntot + i]};
            double xx[3] = {xi_[0], xi_[1], xi_[2]};
            integrate_one(st, mode, false, F, vv, xx, st.seed, (uint64_t)tg, step);
            for (int a = 0; a < 3; ++a) B.v[a * ntot + i] = vv[a];
            if (mode == MODE_LAST) {
                for (int a = 0; a < 3; ++a) B.Fst[a * ntot + i] = F[a];
            } else {
                double *Xn = B.x[cur ^ 1];
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    Xn[a * ntot + i] = xx[a];
                    double dd = xx[a] - B.xref[a * ntot + i];
                    d2 += dd * dd;
                }
                if (d2 > R.disp2) mv = true;
            }
        }
    }
    if (bad) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_NONFINITE);
    if (mv) moved = 1;
    if (THERMO) {
        int wv = threadIdx.x / VBC_WAVE, ln = threadIdx.x % VBC_WAVE;
        for (int k = 0; k < 8; ++k) {
            double v = wave_sum(acc[k]);
            if (ln == 0) red[k][wv] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (moved) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_REBUILD);
    }
    if (THERMO && threadIdx.x < 8) {
        int nw = blockDim.x / VBC_WAVE;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
        B.part[(size_t)b * 8 + threadIdx.x] = s;
    }
}

// Opening half-kick and drift of the first step of a call, from the forces kept in Fst.
__global__ void k_kick_drift(Buffers B, int nrep, int64_t ntot, int cur, StepArgs st)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    int r = rep_of_particle(B.reps, nrep, i);
    const RepDev &R = B.reps[r];
    double F[3], v[3], x[3];
    for (int a = 0; a < 3; ++a) {
        F[a] = B.Fst[a * ntot + i];
        v[a] = B.v[a * ntot + i];
        x[a] = B.x[cur][a * ntot + i];
    }
    integrate_one(st, MODE_MID, true, F, v, x, st.seed, (uint64_t)B.tag[i],
                  B.step[r] + st.step_off);
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        B.v[a * ntot + i] = v[a];
        B.x[cur ^ 1][a * ntot + i] = x[a];
        double dd = x[a] - B.xref[a * ntot + i];
        d2 += dd * dd;
    }
    if (d2 > R.disp2) atomicOr(&B.flags[r], (uint32_t)VBC_FLAG_REBUILD);
}

// Per-replica totals from the per-brick partial sums, in brick order.
__global__ void k_reduce(Buffers B, int nrep, double *__restrict__ UW)
{
    int r = blockIdx.x;
    const RepDev &R = B.reps[r];
    __shared__ double red[8][1024 / VBC_WAVE];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // fixed assignment of bricks to threads, then a fixed-order combine
    for (int b = threadIdx.x; b < R.nbrick; b += blockDim.x)
        for (int k = 0; k < 8; ++k) acc[k] += B.part[(size_t)(R.b_off + b) * 8 + k];
    int wv = threadIdx.x / VBC_WAVE, ln = threadIdx.x % VBC_WAVE;
    for (int k = 0; k < 8; ++k) {
        double v = wave_sum(acc[k]);
        if (ln == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x / VBC_WAVE); ++w) s += red[threadIdx.x][w];
        UW[r * 8 + threadIdx.x] = s;
    }
}

// Export the list of one replica as tag pairs.
__global__ void k_export_nlist(Buffers B, Launch P, int rep, int32_t *__restrict__ pairs,
                               int64_t cap, unsigned long long *__restrict__ count)
{
    extern __shared__ __align__(32) unsigned char smem[];
    __shared__ StageHdr S;
    int b = blockIdx.x;
    const RepDev &R = B.reps[rep];
    if (b >= R.nbrick) return;
    int nh_cap = (P.nh_max + 3) & ~3;
    StageTabs T = carve_tabs(smem, nh_cap);
    stage_tables(R, b, B, S, T, 1 << 30);
    for (int t = threadIdx.x; t < S.n_own; t += blockDim.x) {
        int64_t i = S.own_start + t;
        int nn = B.nn[i];
        for (int s = 0; s < nn; ++s) {
            int u = B.nl[(size_t)s * P.ntot + i];
            int64_t src;
            int w;
            stage_source(S, T, u, src, w);
            unsigned long long k = atomicAdd(count, 1ull);
            if ((int64_t)k < cap) {
                pairs[2 * k] = B.tag[i];
                pairs[2 * k + 1] = B.tag[src];
            }
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

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

size_t lds_bytes_nlist(const Launch &P) { return tabs_bytes(P) + (size_t)P.stage_cap * 24; }
size_t lds_bytes_count(const Launch &P)
{
    return tabs_bytes(P) + (size_t)P.stage_cap * (P.precision == VBC_FP64 ? 32 : 16);
}
size_t lds_bytes_embed(const Launch &P)
{
    return tabs_bytes(P) + (size_t)P.stage_cap * (P.precision == VBC_FP64 ? 40 : 20);
}
size_t lds_bytes_force(const Launch &P)
{
    return tabs_bytes(P) + (size_t)P.stage_cap * (P.precision == VBC_FP64 ? 48 : 24);
}

hipError_t launch_set_state(const Buffers &B, const Launch &P, int rep_lo, int rep_hi,
                            const double *x, const double *v, const int32_t *type,
                            uint64_t step0, hipStream_t s, int64_t n_in, int64_t in_off)
{
    if (n_in <= 0) return hipSuccess;
    k_set_state<<<blocks_for(n_in, 256), 256, 0, s>>>(B, P.nrep, P.ntot, rep_lo, rep_hi, in_off,
                                                       n_in, x, v, type, step0);
    return hipGetLastError();
}

hipError_t launch_get_state(const Buffers &B, const Launch &P, int cur, int rep_lo, int rep_hi,
                            double *x, double *v, hipStream_t s, int64_t n_out, int64_t out_off)
{
    if (n_out <= 0) return hipSuccess;
    k_get_state<<<blocks_for(n_out, 256), 256, 0, s>>>(B, P.nrep, P.ntot, cur, rep_lo, rep_hi,
                                                        out_off, n_out, x, v);
    return hipGetLastError();
}

hipError_t launch_flags(const Buffers &B, const Launch &P, uint32_t bits, bool set, hipStream_t s)
{
    if (set)
        k_flags_or<<<blocks_for(P.nrep, 64), 64, 0, s>>>(B, P.nrep, bits);
    else
        k_flags_clear<<<blocks_for(P.nrep, 64), 64, 0, s>>>(B, P.nrep, bits);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Buffers &B, const Launch &P, int cur, hipStream_t s)
{
    k_bin<<<blocks_for(P.ntot, 256), 256, 0, s>>>(B, P.nrep, P.ntot, cur);
    k_scan<<<P.nrep, 1024, 0, s>>>(B, P.nrep);
    k_scatter<<<blocks_for(P.ntot, 256), 256, 0, s>>>(B, P.nrep, P.ntot);
    k_cellsort<<<blocks_for(P.ncell_tot, 128), 128, 0, s>>>(B, P.nrep, P.ntot, P.ncell_tot, cur);
    k_nlist<<<brick_grid(P.nbrick_tot), P.block, lds_bytes_nlist(P), s>>>(B, P, cur);
    return hipGetLastError();
}

hipError_t launch_count(const Buffers &B, const Launch &P, int cur, double *n_out, hipStream_t s)
{
    size_t lds = lds_bytes_count(P);
    unsigned g = brick_grid(P.nbrick_tot);
    bool multi = P.ntypes_max > 1;
    if (P.precision == VBC_FP64) {
        if (multi) k_count<double, true><<<g, P.block, lds, s>>>(B, P, cur, n_out);
        else k_count<double, false><<<g, P.block, lds, s>>>(B, P, cur, n_out);
    } else {
        if (multi) k_count<float, true><<<g, P.block, lds, s>>>(B, P, cur, n_out);
        else k_count<float, false><<<g, P.block, lds, s>>>(B, P, cur, n_out);
    }
    return hipGetLastError();
}

hipError_t launch_embed(const Buffers &B, const Launch &P, int cur, hipStream_t s)
{
    size_t lds = lds_bytes_embed(P);
    unsigned g = brick_grid(P.nbrick_tot);
    bool multi = P.ntypes_max > 1;
    if (P.precision == VBC_FP64) {
        if (multi) k_embed<double, true><<<g, P.block, lds, s>>>(B, P, cur);
        else k_embed<double, false><<<g, P.block, lds, s>>>(B, P, cur);
    } else {
        if (multi) k_embed<float, true><<<g, P.block, lds, s>>>(B, P, cur);
        else k_embed<float, false><<<g, P.block, lds, s>>>(B, P, cur);
    }
    return hipGetLastError();
}

template <class Real, bool MULTI>
static void launch_force_t(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                           const StepArgs &st, double *F_out, double *e_out, hipStream_t s)
{
    size_t lds = lds_bytes_force(P);
    unsigned g = brick_grid(P.nbrick_tot);
    if (thermo)
        k_force<Real, MULTI, true><<<g, P.block, lds, s>>>(B, P, cur, (int)mode, st, F_out, e_out);
    else
        k_force<Real, MULTI, false><<<g, P.block, lds, s>>>(B, P, cur, (int)mode, st, F_out, e_out);
}

hipError_t launch_force(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                        const StepArgs &st, double *F_out, double *e_out, hipStream_t s)
{
    bool multi = P.ntypes_max > 1;
    if (P.precision == VBC_FP64) {
        if (multi) launch_force_t<double, true>(B, P, cur, mode, thermo, st, F_out, e_out, s);
        else launch_force_t<double, false>(B, P, cur, mode, thermo, st, F_out, e_out, s);
    } else {
        if (multi) launch_force_t<float, true>(B, P, cur, mode, thermo, st, F_out, e_out, s);
        else launch_force_t<float, false>(B, P, cur, mode, thermo, st, F_out, e_out, s);
    }
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
    k_kick_drift<<<blocks_for(P.ntot, 256), 256, 0, s>>>(B, P.nrep, P.ntot, cur, st);
    return hipGetLastError();
}

hipError_t launch_advance(const Buffers &B, const Launch &P, uint64_t nsteps, hipStream_t s)
{
    k_advance<<<blocks_for(P.nrep, 64), 64, 0, s>>>(B, P.nrep, nsteps);
    return hipGetLastError();
}

hipError_t launch_export_nlist(const Buffers &B, const Launch &P, int rep, int nbrick,
                               int32_t *pairs, int64_t cap, int64_t *count, hipStream_t s)
{
    unsigned long long *c = (unsigned long long *)count;
    k_zero_u64<<<1, 1, 0, s>>>(c);
    if (nbrick > 0)
        k_export_nlist<<<nbrick, P.block, tabs_bytes(P), s>>>(B, P, rep, pairs, cap, c);
    return hipGetLastError();
}

}  // namespace vbc
