/*
 * vbc.h -- C ABI of libvbc.so, the MI355X (gfx950) hot path of the valency-bounding
 * correction (VBC): Dmitriev, Gupta & Goloborodko, "Valency-bounding correction
 * potential for coarse-grained molecular dynamics simulations", arXiv 2609.07842.
 *
 * The library evaluates, for one or more independent periodic particle systems
 * ("replicas") resident in GPU memory:
 *   U = sum_{i<j} [ V_r(r_ij) + Psi(n_i, n_j) V_a(r_ij) ]          Section 2, eq. (Vhat)
 *   n_i = sum_{j != i} omega(r_ij, r_l, r_h)                          eq. (counter)
 *   Psi = omega(n_i, f-delta, f-delta+1) omega(n_j, f-delta, f-delta+1)   eq. (Psi), (Psidelta)
 * with the polynomial soft-core V_r, V_a of eq. (softcore), the smooth step omega of
 * eq. (omega), and the forces -grad U including the chain-rule terms through dPsi/dn.
 *
 * Conventions shared by every entry point:
 *  - Every function returns a vbc_status; nothing throws across the ABI.  On error
 *    vbc_last_error(h) returns a message owned by the handle (valid until the next call).
 *  - "Device" pointers are HIP device memory owned by the caller.  The library allocates
 *    no device memory at all: all of its state lives in the caller-provided workspace
 *    (size from vbc_workspace_size), which must stay alive until vbc_destroy.
 *  - Calls that take a hipStream_t are asynchronous on that stream.  The set-up and
 *    read-back calls (vbc_create, vbc_pool_create, vbc_check, vbc_get_stats,
 *    vbc_profile_read, vbc_stamps, vbc_stamps_read) synchronise or clear memory with
 *    copies; vbc_admit uploads a descriptor with one host-to-device copy; the others
 *    launch kernels only.  Conditions detected on the GPU (list or staging
 *    overflow, non-finite coordinates) are latched per replica in the workspace and
 *    reported by vbc_check, which synchronises the stream.
 *  - Per-particle caller arrays are structure-of-arrays over "caller order": replica r
 *    occupies indices [o_r, o_r + N_r); inside a replica, index = tag, the particle's
 *    position in the arrays given to vbc_set_state or vbc_admit.  A 3-vector array holds
 *    all x components, then all y, then all z, with stride Ntot.  For a handle made by
 *    vbc_create, o_r = N_0 + ... + N_{r-1} and Ntot = sum of N_r; for a pool
 *    (vbc_pool_create), Ntot = max_particles and o_r comes from vbc_replica_info.
 *  - Calls on one handle must be ordered: issue them on one stream, or synchronise.
 *  - Units: unit masses; energies in the units of E_r, E_a; kT in the same units.
 */
#ifndef VBC_H
#define VBC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vbc_status;
enum {
    VBC_OK = 0,
    VBC_ERR_ARG = 1,            /* invalid argument or parameter set */
    VBC_ERR_BOX = 2,            /* box shorter than 2 x (cutoff + skin), or fewer than 3 cells */
    VBC_ERR_NLIST_OVERFLOW = 3, /* a particle had more list neighbours than k_max */
    VBC_ERR_NONFINITE = 4,      /* a coordinate became NaN or infinite */
    VBC_ERR_HIP = 5,            /* a HIP runtime call failed */
    VBC_ERR_CAPACITY = 6,       /* a cell brick held more particles than the staging capacity,
                                   or the workspace is too small */
    VBC_ERR_UNIMPLEMENTED = 7,
    VBC_ERR_STATE = 8           /* call out of order (e.g. no state set yet) */
};

/* Bits of the per-replica flag word reported by vbc_check. */
enum {
    VBC_FLAG_REBUILD = 1u,         /* internal: list rebuild pending */
    VBC_FLAG_NLIST_OVERFLOW = 2u,
    VBC_FLAG_STAGE_OVERFLOW = 4u,
    VBC_FLAG_NONFINITE = 8u,
    VBC_FLAG_LOST = 16u            /* a particle moved further than one cell between two list
                                      builds (unstable dynamics); reported as VBC_ERR_NONFINITE */
};

/* Parameters of one type pair (Section 2, eq. (softcore); eq. (counter); eq. (Psidelta)).
 * Requires 0 <= E_r, 0 <= E_a, 0 < r_r < r_a, 0 < r_l < r_h.  f and delta are real. */
typedef struct {
    double E_r, r_r; /* repulsive core height and range */
    double E_a, r_a; /* attractive well depth and outer range (well centred at (r_a+r_r)/2) */
    double r_l, r_h; /* counting radii: a neighbour counts 1 below r_l, 0 above r_h */
    double f, delta; /* valency cap and switching shift (threshold f - delta) */
} vbc_pair_params;

enum { VBC_FP64 = 0, VBC_FP32_MIXED = 1 };

/* One replica (independent periodic system).  Host memory; copied by vbc_create. */
typedef struct {
    int64_t n;                      /* particles, >= 1 */
    double L[3];                    /* orthorhombic periodic box edges */
    int32_t ntypes;                 /* 1..4 particle types */
    const vbc_pair_params *params;  /* ntypes x ntypes row-major, must be symmetric */
    const uint32_t *count_mask;     /* ntypes words: bit u of word t set => a particle of type
                                       t counts neighbours of type u; NULL = all count all */
    double skin;                    /* neighbour-list buffer added to the largest cutoff */
    int32_t chain_len;              /* > 1: tags form chains of this many consecutive beads
                                       joined by harmonic bonds; 0 = no bonds */
    double k_bond, r0_bond;         /* bond energy k/2 (r - r0)^2 */
    uint64_t seed;                  /* added (mod 2^64) to the integrator's seed to give this
                                       replica's Langevin noise key */
    int32_t excl_span;              /* with chains: beads of one chain at most excl_span apart
                                       along it neither count each other nor attract (their
                                       soft-core repulsion stays); 0 = no exclusions.  With
                                       stickers every s-th bead, excl_span = s forbids binding
                                       between stickers adjacent along the backbone
                                       (Section 6.1).  Needs stage_cap <= 32767. */
} vbc_replica_desc;

/* Layout and launch knobs (0 = automatic).  None of them changes a result beyond the
 * rounding of sums. */
typedef struct {
    int32_t precision;   /* VBC_FP64 or VBC_FP32_MIXED (FP32 pair arithmetic, FP64
                            counts, switching, integration and reductions) */
    int32_t k_max;       /* neighbour-list slots per particle */
    int32_t brick;       /* cells per edge of the cell brick one workgroup owns (1..6) */
    int32_t block;       /* threads per workgroup for brick kernels (64..1024, multiple of 64) */
    int32_t stage_cap;   /* particles staged in LDS per brick (own + halo) */
    double rho_max;      /* > 0: size slots per brick, staging and k_max so that local
                            number densities up to rho_max fit anywhere (clustering or phase
                            separation); 0 = margins around the mean density only */
} vbc_options;

enum { VBC_NVE = 0, VBC_LANGEVIN = 1 };

/* Integrator.  NVE: velocity Verlet.  LANGEVIN: BAOAB splitting with friction gamma at
 * temperature kT; noise from Philox4x32-10 with key = the 32-bit halves of
 * (seed + replica seed) and counter = the halves of step, then of tag; each of the first
 * three output words w is mapped to sqrt(3) (2u - 1), u = (w + 1/2) 2^-32. */
typedef struct {
    int32_t kind;
    double dt, kT, gamma;
    uint64_t seed;
} vbc_integrator;

typedef struct vbc_handle_s *vbc_handle;

/* Bytes of device workspace needed for these replicas and options. */
vbc_status vbc_workspace_size(const vbc_replica_desc *reps, int32_t nrep,
                              const vbc_options *opt, size_t *bytes);

/* Validate the parameters, lay out the workspace d_ws (device, >= the size above, at
 * least 256-byte aligned), upload the static tables on stream s and return a handle.
 * Fails with VBC_ERR_ARG for unphysical or asymmetric parameters and VBC_ERR_BOX for a
 * box that cannot hold the minimum image at the list radius. */
vbc_status vbc_create(const vbc_replica_desc *reps, int32_t nrep, const vbc_options *opt,
                      void *d_ws, size_t ws_bytes, hipStream_t s, vbc_handle *out);
vbc_status vbc_destroy(vbc_handle h);
const char *vbc_last_error(vbc_handle h);

/* Copy positions (device, 3 x N SoA with N = N_rep; any real values, wrapped into the
 * box), velocities (device, same layout, or NULL for zero) and types (device int32 [N], or
 * NULL for type 0) of replica rep into the library, reset its step counter to step0 and
 * mark its list stale.  rep < 0: every live replica, from caller-order arrays (stride
 * Ntot).  The other replicas are left untouched: their next steps give the same results
 * as without this call. */
vbc_status vbc_set_state(vbc_handle h, int32_t rep, const double *d_x, const double *d_v,
                         const int32_t *d_type, uint64_t step0, hipStream_t s);

/* Copy positions (wrapped into [0, L)) and velocities of replica rep (3 x N_rep SoA) or,
 * if rep < 0, of every live replica (caller order, stride Ntot) out.  Either pointer may
 * be NULL. */
vbc_status vbc_get_state(vbc_handle h, int32_t rep, double *d_x, double *d_v, hipStream_t s);

/* Neighbour-list build (Section 5: list at the largest cutoff plus a buffer): wrap
 * positions into the box, bin into cells of edge >= r_list, sort particles by cell
 * (ties by tag), and list for every particle all j != i with minimum-image squared
 * distance < r_list^2, evaluated in FP64 without contraction.  Resets the displacement
 * reference. */
vbc_status vbc_build_nlist(vbc_handle h, hipStream_t s);

/* Pass 1 (Section 2, eq. (counter)): smoothed neighbour counts n_i in FP64, written to
 * d_n (device, [Ntot], caller order) unless NULL.  Rebuilds the list first if stale. */
vbc_status vbc_count(vbc_handle h, double *d_n, hipStream_t s);

/* Passes 1 and 2 (Section 2, two-passes paragraph): forces -grad U into d_F (device,
 * 3 x Ntot SoA, caller order), per-particle energies (half of each pair energy, plus half
 * of each bond energy) into d_e ([Ntot]) and per replica 8 doubles into d_UW
 * ({U, W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz} with W = -sum_{i<j} dU/dr_ij r_ij);
 * each pointer may be NULL. */
vbc_status vbc_force(vbc_handle h, double *d_F, double *d_e, double *d_UW, hipStream_t s);

/* Advance every live replica by nsteps steps of the integrator.  The list is rebuilt on
 * the GPU whenever some particle of a replica has moved more than skin/2 since the last
 * build.  Replicas without stored forces (new state) get them first, each on its own,
 * so that the others are not touched.  Calls of up to 64 steps run as one captured HIP
 * graph launch (captured once per step count, integrator and buffer parity); longer
 * calls replay graphs of 8 steps. */
vbc_status vbc_step(vbc_handle h, int32_t nsteps, const vbc_integrator *it, hipStream_t s);

/* Capture, without launching anything, the step graphs that vbc_step(h, nsteps, it, ...)
 * issued next would launch (the whole-call graph for nsteps <= 64, else the 8-step graph),
 * so that a later call does not pay for the capture.  No state is read or changed.
 * Returns VBC_OK also when graphs are off (kernel timing on). */
vbc_status vbc_step_prepare(vbc_handle h, int32_t nsteps, const vbc_integrator *it);

/* Energy and virial of every step (Section 2, two-passes paragraph: the force pass also
 * gives the energy of eq. (Vhat) and the virial).  enable != 0: from now on the force pass of
 * every step of vbc_step also sums, per brick in FP64, the pair energies (plus bond
 * energies) and the virial {W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz} of the step's new
 * positions (conventions of vbc_force), and reduces them per replica in a fixed order into
 * accumulators in the workspace; enable = 0 stops it.  Either way the accumulators are
 * cleared (on stream s).  vbc_thermo_read synchronises s and returns per replica slot
 * (host array [slots][17]): the number of steps accumulated, the last step's 8 values
 * {U, W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz} and the sums of the 8 over those steps; then
 * it clears the accumulators.  Free slots read 0. */
vbc_status vbc_thermo(vbc_handle h, int32_t enable, hipStream_t s);
vbc_status vbc_thermo_read(vbc_handle h, hipStream_t s, double *out);

/* Synchronise s and report the flag word of each replica slot (host array [nrep] or
 * [max_replicas], may be NULL; 0 for free slots);
 * returns the first error among them (overflow or non-finite) and clears the error bits. */
vbc_status vbc_check(vbc_handle h, hipStream_t s, uint32_t *flags_per_replica);

/* The current neighbour list of replica rep as tag pairs: for every particle i and
 * every listed j, (tag_i, tag_j) into d_pairs (device int32, 2 x cap interleaved); the
 * number of pairs into *d_count (device int64).  Pairs beyond cap are counted, not
 * written.  Test and inspection aid. */
vbc_status vbc_get_nlist(vbc_handle h, int32_t rep, int32_t *d_pairs, int64_t cap,
                         int64_t *d_count, hipStream_t s);

/* Observables of valency control (Section 3): for every particle the number z_i of
 * particles within the attraction range r_a of the pair (the paper's instantaneous bond
 * criterion, r_ij < r_a) and the number p_i within the repulsive core r_r (core
 * penetrations, Section 6.2), decided in FP64 exactly as the plain definition on the
 * positions vbc_get_state returns (minimum image by round-half-even, no contraction).
 * d_z, d_pen: device int32 [Ntot] in caller order, or NULL; d_sums: device int64
 * [slots][3] = {sum of z_i, number of particles with z_i > f (f of the particle's own type
 * pair), sum of p_i} per replica, or NULL.  Rebuilds the list first if it is stale. */
vbc_status vbc_observables(vbc_handle h, int32_t *d_z, int32_t *d_pen, int64_t *d_sums,
                           hipStream_t s);

/* Clusters of the bond graph (Section 3, "Saturation and connectivity", "Cyclisation" and
 * "Cluster-size distributions"): particles i and j are bonded when r_ij < r_a of the pair,
 * the criterion of vbc_observables decided the same way; clusters are the connected
 * components of the bonds within each replica.  A cluster of s particles and e bonds
 * carries a loop (is cyclic) when e >= s; otherwise it is a tree (e = s - 1).
 *   d_scratch      device memory of vbc_cluster_scratch_size bytes, 256-byte aligned, owned
 *                  by the caller; its contents are overwritten (no state is kept)
 *   d_label        device int32 [Ntot] in caller order, or NULL: the smallest tag (replica-
 *                  local) of the particle's cluster
 *   d_stats        device int64 [slots][5] per replica, or NULL: number of clusters, size of
 *                  the largest (P_inf = largest / N), particles in cyclic clusters (x_cyc =
 *                  that / N), bonds, cyclic clusters
 *   d_hist         device int64 [slots][2][hist_len], or NULL: row 0 counts every cluster by
 *                  size, row 1 the acyclic ones; index s < hist_len holds size s and index 0
 *                  the clusters of size >= hist_len
 * Rebuilds the list first if it is stale.  Asynchronous on s; returns VBC_ERR_ARG for a
 * missing or small scratch, or with d_hist given for hist_len outside 1..2^24 or
 * 2 x slots x hist_len of 2^31 or more. */
vbc_status vbc_cluster_scratch_size(vbc_handle h, size_t *bytes);
vbc_status vbc_clusters(vbc_handle h, void *d_scratch, size_t scratch_bytes, int32_t *d_label,
                        int64_t *d_stats, int64_t *d_hist, int32_t hist_len, hipStream_t s);

/* vbc_clusters without caller scratch, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * outputs, arguments and errors as vbc_clusters; the scratch is a fixed array of
 * VBC_CLUSTERS_NOALLOC_BYTES that the library holds in every GPU it runs on until the
 * process ends (its address is looked up on the first call on a device).  The call
 * allocates and frees nothing.  Returns VBC_ERR_CAPACITY when the handle needs more
 * scratch than that (vbc_cluster_scratch_size: 20 bytes per particle slot, about 1.6 x 10^6
 * slots fit).  All calls on one GPU share the array, which keeps the last call's contents
 * (each call rewrites what it reads first): calls that overlap in time on one GPU, on
 * different streams or handles, race and give wrong results, so order them. */
#define VBC_CLUSTERS_NOALLOC_BYTES (32u << 20)
vbc_status vbc_clusters_noalloc(vbc_handle h, int32_t *d_label, int64_t *d_stats, int64_t *d_hist,
                                int32_t hist_len, hipStream_t s);

/* Bond lifetimes (Section 4, "Bond lifetimes"): one sample of a tracker that follows every
 * bond (r_ij < r_a of the pair, the criterion of vbc_observables) from the first sample at
 * which it is seen to the first sample without it, at the replicas' current step counters.
 *   d_state        device memory of vbc_bond_track_size bytes, 256-byte aligned, owned by the
 *                  caller and kept between calls: per caller index the count of stored
 *                  partners, their tags and the steps their bonds were first seen
 *   max_partners   bonds stored per particle, 1..64; bonds that do not fit are counted
 *   reset          nonzero: start tracking from the current bonds (their births unknown)
 *                  and zero d_hist and d_stats; call it after set_state or an admission
 *   d_hist         device int64 [slots][hist_len], or NULL: completed bonds (first seen at a
 *                  sample, gone at a later one) by lifetime in steps / bin_steps; the last bin
 *                  holds the longer ones
 *   d_stats        device int64 [slots][5], or NULL: bonds formed, bonds broken with a
 *                  lifetime, bonds broken that existed at the reset, bonds that did not fit,
 *                  bonds summed over the samples
 * Each bond is counted once, at its end with the smaller tag.  d_hist and d_stats add up
 * over the calls after a reset.  Rebuilds the list first if it is stale.  Asynchronous on s;
 * returns VBC_ERR_ARG for a missing, small or misaligned state or bad sizes. */
vbc_status vbc_bond_track_size(vbc_handle h, int32_t max_partners, size_t *bytes);
vbc_status vbc_bond_track(vbc_handle h, void *d_state, size_t state_bytes, int32_t max_partners, int32_t reset,
                          int64_t *d_hist, int32_t hist_len, int64_t bin_steps, int64_t *d_stats, hipStream_t s);

/* Layout actually chosen (after automatic choices): k_max, brick edge, block, stage_cap. */
vbc_status vbc_get_options(vbc_handle h, vbc_options *out);

/* Change the knobs that do not touch the workspace layout, for the autotuner: block (the
 * workgroup size of the brick kernels; 0 = keep).  Results do not change beyond the
 * rounding of the per-brick energy/virial partial sums (forces and trajectories are
 * bit-identical).  k_max, brick and stage_cap must be 0 or equal to the current values
 * (VBC_ERR_UNIMPLEMENTED otherwise: they set the layout); precision must match.  Captured
 * step graphs are dropped and recaptured on the next vbc_step. */
vbc_status vbc_tune_set(vbc_handle h, const vbc_options *t);

/* Counters kept per replica on the GPU (read with vbc_get_stats, which synchronises s):
 * list builds so far, list entries after the last build (sum over particles), ordered
 * pairs inside the interaction cutoff summed over the count passes that sample them
 * (every pass of vbc_count and vbc_force, and the steps of vbc_step whose index inside
 * the call is a multiple of 8), and the number of those passes.  pair_evals / evals is
 * the mean number of pair evaluations per pass. */
typedef struct {
    uint64_t builds, list_entries, pair_evals, evals;
} vbc_stats;
vbc_status vbc_get_stats(vbc_handle h, hipStream_t s, vbc_stats *out /* host [slots] */);

/* Kernel timing with HIP events that each launch of a kernel class records from its own
 * dispatches (hipExtLaunchKernel: the start of the class's first kernel and the end of its
 * last, with no marker packets between them), on the launch stream, for at most
 * max_launches launches per class (enable = 0 switches it off).
 * Classes: 0 list build (its five kernels together), 1 count, 2 embed, 3 force,
 * 4 first-step kick, 5 reductions.  vbc_profile_read synchronises s and returns, per
 * class, the summed milliseconds and the number of timed launches, then resets them. */
enum { VBC_K_BUILD = 0, VBC_K_COUNT = 1, VBC_K_EMBED = 2, VBC_K_FORCE = 3, VBC_K_KICK = 4,
       VBC_K_REDUCE = 5, VBC_NK = 6 };
vbc_status vbc_profile(vbc_handle h, int32_t enable, int32_t max_launches);
vbc_status vbc_profile_read(vbc_handle h, hipStream_t s, double *ms /* [VBC_NK] */,
                            int64_t *launches /* [VBC_NK] */);

/* ---- Replica pools: continuous batching of independent systems ------------------------
 * A pool is a handle of fixed capacity into which replicas are admitted and from which
 * they retire while others keep running; every launch covers the whole capacity (bricks
 * of free or retired replicas exit at once), so the captured step graphs stay valid as the
 * replica set changes.  The use case is the paper's own way of working: its results are
 * sweeps over many independent state points (valency, temperature, density, well depth;
 * Sections 3 to 5), each a separate simulation. */

/* Fixed capacity of a pool. */
typedef struct {
    int32_t max_replicas;   /* replica slots */
    int32_t max_types;      /* 1..4 particle types per replica */
    int64_t max_particles;  /* particles over all live replicas (caller-order index space) */
    int64_t max_slots;      /* particle slots; a replica takes bricks x bcap of them */
    int32_t max_bricks;     /* cell bricks (one workgroup each) */
    int32_t max_cells;
    int32_t max_bcap;       /* slots per brick of any replica (>= 64) */
    int32_t chains;         /* nonzero: replicas may carry bonded chains */
} vbc_pool_caps;

/* What one replica takes from a workspace (vbc_replica_footprint). */
typedef struct {
    int64_t slots;          /* particle slots (bricks x bcap) */
    int32_t bricks, cells;
    int32_t bcap;           /* slots per brick */
    int32_t k_max;          /* automatic list length for this replica alone */
    int32_t stage_cap;      /* automatic staging capacity for this replica alone */
    int32_t brick;          /* brick edge actually used (cells) */
    size_t bytes;           /* workspace bytes it occupies with these options (k_max and
                               stage_cap of opt, or the automatic ones if 0) */
} vbc_footprint;

/* Layout of one replica and its share of a workspace: the basis of admission by memory
 * footprint.  No device access. */
vbc_status vbc_replica_footprint(const vbc_replica_desc *d, const vbc_options *opt,
                                 vbc_footprint *out);

/* Bytes of device workspace for a pool.  opt->k_max and opt->stage_cap must be set (a pool
 * has no replicas to derive them from); block defaults to 256, brick as for vbc_create. */
vbc_status vbc_pool_workspace_size(const vbc_pool_caps *caps, const vbc_options *opt,
                                   size_t *bytes);

/* Make an empty pool in d_ws (device, >= the size above, 256-byte aligned), clearing it
 * synchronously on s. */
vbc_status vbc_pool_create(const vbc_pool_caps *caps, const vbc_options *opt, void *d_ws,
                           size_t ws_bytes, hipStream_t s, vbc_handle *out);

/* Admit a replica with its initial state (as vbc_set_state with rep = the new index;
 * arrays of this replica only, stride N) and return its index in *rep.  Stream-ordered
 * after earlier work on s; the other replicas are not touched.  VBC_ERR_CAPACITY if no
 * slot or no contiguous range of slots, bricks, cells or particle indices is free, if
 * the replica needs a larger brick capacity, k_max or stage_cap than the pool has, or if
 * its count mask leaves out a type it has and the pool was made with max_types = 1 and
 * no chains (such a pool runs the one-type kernels, which count every neighbour). */
vbc_status vbc_admit(vbc_handle h, const vbc_replica_desc *d, const double *d_x,
                     const double *d_v, const int32_t *d_type, uint64_t step0, hipStream_t s,
                     int32_t *rep);

/* Free replica rep's slot and ranges (stream-ordered: work already issued on s still sees
 * it).  Read its state out first. */
vbc_status vbc_retire(vbc_handle h, int32_t rep, hipStream_t s);

/* Particles and caller-order offset of replica rep (0, 0 for a free slot). */
vbc_status vbc_replica_info(vbc_handle h, int32_t rep, int64_t *n, int64_t *caller_offset);

/* Step time stamps: when enabled, every step of vbc_step ends with a one-thread kernel that
 * writes the device's constant-rate clock into a ring of 65536 entries in the workspace.
 * vbc_stamps (re)starts the ring; vbc_stamps_read synchronises s, returns the last
 * min(written, 65536, cap) stamps in order and the clock rate in Hz, and restarts it.
 * Successive stamps bound each step's latency from end to end. */
vbc_status vbc_stamps(vbc_handle h, int32_t enable, hipStream_t s);
vbc_status vbc_stamps_read(vbc_handle h, hipStream_t s, uint64_t *out, int64_t cap, int64_t *n,
                           double *hz);

#ifdef __cplusplus
}
#endif
#endif /* VBC_H */
