// vbc_internal.h -- device-side data layout of libvbc (gfx950).
//
// Particles of every replica live in one flat index space, sorted per replica by cell
// rank.  Cells are ranked brick-major: a "brick" is a block of up to bd^3 cells owned by
// one workgroup, and the cells of one brick have consecutive ranks, so the particles a
// workgroup owns are one contiguous range.  A workgroup stages its own particles and the
// one-cell halo around its brick in LDS; the neighbour list stores, per particle, 16-bit
// indices into that staging order.
#pragma once
#include <stdint.h>

#include "../../include/vbc.h"

namespace vbc {

constexpr int MAXT = 4;          // particle types per replica
constexpr int MAX_BRICK = 6;     // cells per brick edge
constexpr int NH_MAX = (MAX_BRICK + 2) * (MAX_BRICK + 2) * (MAX_BRICK + 2);

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
    int32_t attract;       // E_a > 0
    int32_t pad;
};

struct RepDev {
    int64_t p_off;         // first internal (sorted) index of this replica
    int64_t n;             // particles
    int64_t o_off;         // first caller-order index
    int32_t c_off;         // offset into cell_rank (ncell entries per replica)
    int32_t cs_off;        // offset into cell_start (ncell + 1 entries per replica)
    int32_t b_off;         // first global brick id
    int32_t nbrick;
    int32_t ncell;
    int32_t nc[3];         // cells per axis
    int32_t bd[3];         // brick edge per axis (cells)
    int32_t nb[3];         // bricks per axis
    int32_t ntypes;
    int32_t chain_len;
    uint32_t mask[MAXT];
    double L[3], h[3];
    double rc2;            // largest interaction cutoff squared
    double rlist2;         // list radius squared (FP64, exact comparison)
    double disp2;          // squared displacement that triggers a rebuild ((skin/2)^2)
    double k_bond, r0_bond;
    PairDev pair[MAXT * MAXT];
};

// Pointers into the caller's workspace.
struct Buffers {
    RepDev *reps;           // [nrep]
    int32_t *cell_rank;     // [sum ncell]  cell linear index -> brick-major rank
    int32_t *brick_rank0;   // [nbrick_tot] rank of a brick's first cell
    int32_t *cell_cnt;      // [sum ncell]  binning counters (kept zero between builds)
    int64_t *cell_start;    // [sum (ncell+1)] internal index of each rank's first particle
    double *x[2];           // positions, SoA [3][ntot], double-buffered by step parity
    double *v;              // velocities SoA [3][ntot]
    double *Fst;            // forces kept between calls SoA [3][ntot]
    double *xref;           // positions at the last build SoA [3][ntot]
    int32_t *tag;           // [ntot] tag of each internal slot
    int32_t *type;          // [ntot]
    int32_t *pcell;         // [ntot] cell rank of each particle at the last build
    int64_t *inv;           // [ntot] replica-local tag -> internal index (by p_off + tag)
    // rebuild scratch
    int32_t *slot;          // [ntot]
    int32_t *perm;          // [ntot]
    double *xs;             // [3][ntot]
    double *vs;             // [3][ntot]
    int32_t *tags;          // [ntot]
    int32_t *types;         // [ntot]
    int32_t *pcs;           // [ntot]
    // list
    uint16_t *nl;           // [k_max][ntot]
    uint16_t *nn;           // [ntot]
    // pass outputs
    double *nd;             // [ntot] counts (FP64)
    void *sA;               // [ntot] (s or n, A) as float2 / double2
    uint8_t *win;           // [nbrick_tot] brick holds a particle inside a switching window
    double *part;           // [nbrick_tot][8] per-brick energy/virial partial sums
    uint32_t *flags;        // [nrep]
    uint64_t *step;         // [nrep] step counter (noise counter)
};

struct Launch {
    int nrep;
    int64_t ntot;
    int32_t ncell_tot;      // sum ncell
    int32_t ncs_tot;        // sum (ncell + 1)
    int32_t nbrick_tot;
    int32_t k_max;
    int32_t block;
    int32_t stage_cap;
    int32_t nh_max;         // max halo-grid cells of any brick
    int32_t ntypes_max;
    int32_t any_chains;
    int32_t precision;
};

enum Mode { MODE_EVAL = 0, MODE_MID = 1, MODE_LAST = 2 };

struct StepArgs {
    int kind;               // VBC_NVE / VBC_LANGEVIN
    double dt, hdt;
    double c1, c2s;         // Langevin O-step coefficients
    uint64_t seed;
    uint64_t step_off;      // added to the per-replica step counter
};

// host-side launchers (vbc_kernels.hip)
hipError_t launch_set_state(const Buffers &B, const Launch &P, int rep_lo, int rep_hi,
                            const double *x, const double *v, const int32_t *type,
                            uint64_t step0, hipStream_t s, int64_t n_in, int64_t in_off);
hipError_t launch_get_state(const Buffers &B, const Launch &P, int cur, int rep_lo, int rep_hi,
                            double *x, double *v, hipStream_t s, int64_t n_out, int64_t out_off);
hipError_t launch_flags(const Buffers &B, const Launch &P, uint32_t bits, bool set, hipStream_t s);
hipError_t launch_rebuild(const Buffers &B, const Launch &P, int cur, hipStream_t s);
hipError_t launch_count(const Buffers &B, const Launch &P, int cur, double *n_out, hipStream_t s);
hipError_t launch_embed(const Buffers &B, const Launch &P, int cur, hipStream_t s);
hipError_t launch_force(const Buffers &B, const Launch &P, int cur, Mode mode, bool thermo,
                        const StepArgs &st, double *F_out, double *e_out, hipStream_t s);
hipError_t launch_reduce(const Buffers &B, const Launch &P, double *UW, hipStream_t s);
hipError_t launch_kick_drift(const Buffers &B, const Launch &P, int cur, const StepArgs &st,
                             hipStream_t s);
hipError_t launch_advance(const Buffers &B, const Launch &P, uint64_t nsteps, hipStream_t s);
hipError_t launch_export_nlist(const Buffers &B, const Launch &P, int rep, int nbrick,
                               int32_t *pairs, int64_t cap, int64_t *count, hipStream_t s);
size_t lds_bytes_nlist(const Launch &P);
size_t lds_bytes_count(const Launch &P);
size_t lds_bytes_embed(const Launch &P);
size_t lds_bytes_force(const Launch &P);

}  // namespace vbc
