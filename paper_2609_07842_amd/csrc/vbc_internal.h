// vbc_internal.h -- device-side data layout of libvbc (gfx950).
//
// Space is cut into cells of edge >= the list radius, and cells into "bricks" of up to
// bd^3 cells; one workgroup owns one brick.  The workspace is a pool of fixed capacity
// (replica descriptors, bricks, cells, particle slots, caller-order indices); a replica
// takes a contiguous range of each, and a table gives the owner of every brick (-1 for a
// free one), so replicas can enter and leave without changing any launch shape.  Every brick has a fixed number of particle
// slots (bcap), so a replica's particles live in nbrick * bcap slots without any global
// prefix sum: brick b of replica r owns slots [p_off + b * bcap, p_off + b * bcap + bcnt[b]),
// sorted by cell (cells in x-fastest order inside the brick) and by tag inside a cell.
// A workgroup stages its own particles and the one-cell halo around its brick in LDS in a
// brick-local frame; the neighbour list stores per particle 16-bit indices into that
// staging order, in chunks of eight (one 16-byte load per chunk).
#pragma once
#include <stdint.h>

#include "../../include/vbc.h"

namespace vbc {

constexpr int MAXT = 4;          // particle types per replica
constexpr int MAX_BRICK = 6;     // cells per brick edge
constexpr int NH_MAX = (MAX_BRICK + 2) * (MAX_BRICK + 2) * (MAX_BRICK + 2);
constexpr int CHUNK = 8;         // list entries per 16-byte chunk
constexpr int MAX_REPLICAS = 1024;  // replica slots of one handle

// Derived constants of one type pair.  Everything the kernels need is precomputed on
// the host in FP64 from vbc_pair_params.
struct PairDev {
    double E_r, r_r, E_a, r_a, r_l, r_h;
    double x1, x2;         // switching interval of eq. (Psidelta): f - delta, f - delta + 1
    double rr2, ra2, rl2, rh2;
    double inv_rr2;        // 1 / r_r^2
    double c_r;            // -4 E_r / r_r^2  (V_r'(r)/r = c_r (1 - r^2/r_r^2))
    double m, inv_w;       // well centre (r_a + r_r)/2 and 1 / ((r_a - r_r)/2)
    double c_a;            // 4 E_a / w   (V_a'(r) = c_a u (1 - u^2))
    double inv_dw;         // 1 / (r_h - r_l)
    double c_c;            // -4 / (r_h - r_l)  (c'(r) = c_c u (1 - u^2))
    double f;              // valency
    int32_t attract;       // E_a > 0
    int32_t pad;
};

struct RepDev {
    int64_t p_off;         // first slot of this replica
    int64_t n;             // particles
    int64_t o_off;         // first caller-order index
    int32_t bcap;          // slots per brick
    int32_t c_off;         // offset into the per-cell tables (ncell entries per replica)
    int32_t b_off;         // first global brick id
    int32_t nbrick;
    int32_t ncell;
    int32_t nc[3];         // cells per axis
    int32_t bd[3];         // brick edge per axis (cells)
    int32_t nb[3];         // bricks per axis
    int32_t ntypes;
    int32_t chain_len;
    int32_t excl_span;     // > 0: chain neighbours up to this many beads apart neither count
                           // nor attract each other (list entries carry bit 15)
    uint32_t mask[MAXT];
    double L[3], h[3];
    double rc2;            // largest interaction cutoff squared
    double rlist2;         // list radius squared (FP64, exact comparison)
    double disp2;          // squared displacement that triggers a rebuild ((skin/2)^2)
    double k_bond, r0_bond;
    uint64_t seed;         // added to the integrator's seed: this replica's noise key
    PairDev pair[MAXT * MAXT];
};

// Pointers into the caller's workspace.  [2] = {live, next}: a list build writes the new
// sorted layout into "next" and the list kernel copies each brick into "live".
struct Buffers {
    RepDev *reps;            // [nrep]
    int32_t *brick_rep;      // [nbrick_tot] replica owning each brick, -1 = free
    int32_t *wl[2];          // [nbrick_tot] work lists: live bricks, bricks due for a rebuild
    int32_t *wl_n;           // [2] entries of each work list
    int32_t *cell_rank;      // [sum ncell]  cell linear index -> brick-major rank (static)
    int32_t *brick_rank0;    // [nbrick_tot] rank of a brick's first cell (static)
    int32_t *cstart[2];      // [sum ncell] first slot of each cell (by rank)
    int32_t *ccnt[2];        // [sum ncell] particles in each cell (by rank)
    int32_t *bcnt[2];        // [nbrick_tot] particles in each brick
    int32_t *bfill;          // [nbrick_tot] counters of the full (unsorted-input) build
    double *x[2];            // positions [nslots][3] (the three coordinates of a slot side by
                             // side, so that a cell's particles gathered into a neighbour's
                             // halo are one contiguous run), double-buffered by step parity
    double *v;               // velocities SoA [3][nslots]
    double *Fst;             // forces kept between calls SoA [3][nslots]
    double *xref;            // positions at the last build SoA [3][nslots]
    int32_t *tag;            // [nslots]
    int32_t *type;           // [nslots]
    uint8_t *lcell;          // [nslots] cell of the particle inside its brick
    double *xs;              // next layout: positions [nslots][3]
    double *vs;              // next layout: velocities
    int32_t *tags, *types;   // next layout
    uint8_t *lcells;         // next layout
    int32_t *src;            // [nslots] full build: members of each brick (dense index)
    int32_t *inv;            // [ntot] caller index (o_off + tag) -> slot (kept for chains only)
    int32_t *smap;           // [nbrick_tot][stage_cap] source slot of each staged particle
    uint8_t *wmap;           // [nbrick_tot][stage_cap] packed image shift of each staged particle
    int32_t *stotal;         // [nbrick_tot] staged particles per brick (> stage_cap: overflow)
    uint4 *nl;               // [nchunk][nslots] neighbour list chunks of 8 x uint16
    uint16_t *nn;            // [nslots] list length
    double *nd;              // [nslots] counts (FP64)
    void *sA;                // [nslots] (s or n, A) as float2 / double2
    int32_t *wcnt;           // [nbrick_tot] own particles inside a switching window (last count pass)
    uint16_t *wlst;          // [nslots] per brick: those particles (brick-local index), compact
    double *part;            // [nbrick_tot][8] per-brick energy/virial partial sums
    uint32_t *flags;         // [nrep]
    uint64_t *step;          // [nrep] step counter (noise counter)
    unsigned long long *stats;  // [nrep][4] builds, -, -, count passes
    unsigned long long *bevals; // [nbrick_tot] pair evaluations of each brick, summed over passes
    uint32_t *bentries;         // [nbrick_tot] list entries of each brick at the last build
    unsigned long long *stamps; // [STAMP_CAP] device clock at the end of each stamped step
    unsigned long long *stamp_n; // [1] stamps written so far
    double *thermo;             // [nrep][THERMO_WORDS] steps accumulated, last step's
                                // {U, W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz}, their sums
    int32_t *tpend;             // [nrep] 1: the last time step's per-brick energy and virial
                                // sums (part) are not yet added to thermo
};

constexpr int THERMO_WORDS = 17;

constexpr int STAMP_CAP = 1 << 16;  // power of two

struct Launch {
    int nrep;                // replica slots
    int64_t ntot;            // particles
    int64_t nslots;          // slots (sum nbrick * bcap)
    int32_t ncell_tot;
    int32_t nbrick_tot;
    int32_t b_lo, nb_launch; // bricks one launch covers: [b_lo, b_lo + nb_launch), or
    int32_t list;            // >= 0: the entries of that work list instead
    int32_t k_max;           // multiple of CHUNK
    int32_t nchunk;          // k_max / CHUNK
    int32_t block;
    int32_t stage_cap;
    int32_t nh_max;          // max halo-grid cells of any brick
    int32_t bcap_max;
    int32_t ncb_max;         // max cells of one brick
    int32_t ntypes_max;
    int32_t any_chains;
    int32_t multi;           // general pair path: several types or chain exclusions
    int32_t precision;
    // host side only: the one replica of a fixed single-replica handle (not a pool), whose
    // descriptor the count and force passes then take as a kernel argument; else null
    const RepDev *one;
};

// The replica descriptor as a kernel argument (ONE) or nothing.
template <bool ONE> struct OneRep { int unused; };
template <> struct OneRep<true> { RepDev R; };

// internal flag bits (beyond the public ones in vbc.h)
enum : uint32_t {
    FLAG_FULL = 1u << 8      // next build starts from unsorted (caller-order) input
};

enum Mode { MODE_EVAL = 0, MODE_MID = 1, MODE_LAST = 2 };

struct StepArgs {
    int kind;               // VBC_NVE / VBC_LANGEVIN
    int acc;                // a time step with the energy and virial sums on: the force pass
                            // leaves its per-brick sums for the next count pass (or the call's
                            // closing reduction) to add
    double dt, hdt;
    double c1, c2s;         // Langevin O-step coefficients
    uint64_t seed;
};

// Kernel timing for the profiling mode: while a pair of events is set, the launchers of the
// list build, count, dU/dn and force passes dispatch through hipExtLaunchKernel, which takes
// the events' timestamps from the dispatches themselves (start at the first kernel, stop at
// each, so the last one's end wins), with no marker packets between the kernels.
// launch_events_used() counts the launches that took them since the last set, and
// launch_events_error() returns the first error one of those launches returned.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
int launch_events_used();
hipError_t launch_events_error();

// host-side launchers (vbc_kernels.hip).  Brick kernels cover the bricks
// [P.b_lo, P.b_lo + P.nb_launch), or with P.list >= 0 the work lists that launch_rebuild and
// launch_kick_drift make first.
hipError_t launch_set_state(const Buffers &B, const Launch &P, int cur, int r, int64_t n,
                            const double *x, const double *v, const int32_t *type,
                            int64_t in_off, int64_t in_stride, uint64_t step0, hipStream_t s);
hipError_t launch_get_state(const Buffers &B, const Launch &P, int cur, int r, int64_t nslot,
                            int64_t out_off, int64_t out_stride, double *x, double *v,
                            hipStream_t s);
hipError_t launch_flags(const Buffers &B, int r_lo, int r_n, uint32_t bits, bool set,
                        hipStream_t s);
hipError_t launch_admit(const Buffers &B, int r, int64_t nthreads, hipStream_t s);
hipError_t launch_retire(const Buffers &B, int r, int b_off, int nbrick, hipStream_t s);
hipError_t launch_stamp(const Buffers &B, hipStream_t s);
hipError_t launch_full_build(const Buffers &B, const Launch &P, int cur, int r, int64_t n,
                             hipStream_t s);
hipError_t launch_rebuild(const Buffers &B, const Launch &P, int cur, hipStream_t s);
hipError_t launch_count(const Buffers &B, const Launch &P, int cur, double *n_out, int advance,
                        bool stats, hipStream_t s);
hipError_t launch_embed(const Buffers &B, const Launch &P, int cur, hipStream_t s);
hipError_t launch_force(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                        const StepArgs &st, double *F_out, double *e_out, hipStream_t s);
hipError_t launch_reduce(const Buffers &B, const Launch &P, double *UW, hipStream_t s);
hipError_t launch_thermo_acc(const Buffers &B, const Launch &P, hipStream_t s);
hipError_t launch_thermo_clear(const Buffers &B, int nrep, hipStream_t s);
hipError_t launch_kick_drift(const Buffers &B, const Launch &P, int cur, const StepArgs &st,
                             hipStream_t s);
hipError_t launch_export_nlist(const Buffers &B, const Launch &P, int rep, int nbrick,
                               int32_t *pairs, int64_t cap, int64_t *count, hipStream_t s);
hipError_t launch_observe(const Buffers &B, const Launch &P, int cur, int32_t *z_out,
                          int32_t *pen_out, int64_t *sums, hipStream_t s);

// Scratch of the cluster analysis: five int32 arrays over the slots.
struct ClusterWork {
    int32_t *parent;  // union-find forest; after counting, the root of every particle
    int32_t *size;    // particles per cluster (at the root)
    uint32_t *ends;   // bond ends per cluster (twice its bonds)
    int32_t *mintag;  // smallest caller tag per cluster
    int32_t *z;       // bonds of every particle
};
// State of the bond tracker, by caller index: partner count, then M partner tags and M
// birth steps per particle.
struct BondTrack {
    int32_t *count;   // [ntot]
    int32_t *tags;    // [ntot][M]
    int64_t *births;  // [ntot][M]
    int M;
};
hipError_t launch_bond_track(const Buffers &B, const Launch &P, int cur, const BondTrack &T, int reset,
                             int64_t *hist, int hist_len, int64_t bin_steps, int64_t *stats, hipStream_t s);
hipError_t launch_clusters(const Buffers &B, const Launch &P, int cur, const ClusterWork &W,
                           int32_t *label, int64_t *stats, int64_t *hist, int hist_len, hipStream_t s);
size_t lds_bytes_sort(const Launch &P);
size_t lds_bytes_nlist(const Launch &P);
size_t lds_bytes_count(const Launch &P);
size_t lds_bytes_embed(const Launch &P);
size_t lds_bytes_bonds(const Launch &P);
size_t lds_bytes_force(const Launch &P);

}  // namespace vbc
