/*
 * vbc_oracle.c -- plain FP64 CPU oracle for the valency-bounding correction (VBC)
 * of Dmitriev, Gupta & Goloborodko, "Valency-bounding correction potential for
 * coarse-grained molecular dynamics simulations" (arXiv 2609.07842).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything here is the method's definition evaluated directly:
 *   - all ordered pairs (O(N^2)), no cells, no neighbour list, no blocking;
 *   - FP64 throughout, built with -ffp-contract=off;
 *   - every per-particle sum runs over j in ascending order;
 *   - OpenMP only splits the outer particle loop; each thread writes its own rows,
 *     and totals are summed over i in ascending order afterwards.
 *
 * Where the paper is silent the reading taken is stated next to the code (the
 * same readings are listed in the design notes of the repository).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VBCO_MAXT 8

/* Pair parameters of one type pair, Section 2 eq. (softcore) and eq. (Psidelta):
 * repulsive core E_r, r_r; attractive shell E_a, r_a; counting radii r_l < r_h;
 * valency f and shift delta.  The table is symmetric in the type pair. */
typedef struct {
    double E_r, r_r, E_a, r_a, r_l, r_h, f, delta;
} vbco_pair;

/* ------------------------------------------------------------------------- */
/* Scalar functions                                                           */
/* ------------------------------------------------------------------------- */

/* Smooth step, Section 2.1 eq. (omega): 1 for x <= x1, 0 for x >= x2 and
 * (1 - u^2)^2 with u = (x - x1)/(x2 - x1) in between.  Continuously differentiable. */
double vbco_omega(double x, double x1, double x2)
{
    if (x <= x1) return 1.0;
    if (x >= x2) return 0.0;
    double u = (x - x1) / (x2 - x1);
    double q = 1.0 - u * u;
    return q * q;
}

/* Derivative of eq. (omega) with respect to x: -4 u (1 - u^2) / (x2 - x1) inside
 * the switching interval, zero outside (both one-sided limits vanish at x1, x2). */
double vbco_omega_d(double x, double x1, double x2)
{
    if (x <= x1 || x >= x2) return 0.0;
    double w = x2 - x1;
    double u = (x - x1) / w;
    return -4.0 * u * (1.0 - u * u) / w;
}

/* Repulsive core of eq. (softcore): E_r (1 - (r/r_r)^2)^2 for r < r_r, else 0. */
double vbco_Vr(double r, double E_r, double r_r)
{
    if (r >= r_r) return 0.0;
    double t = r / r_r;
    double q = 1.0 - t * t;
    return E_r * q * q;
}

/* dV_r/dr divided by r, closed form -4 E_r (1 - r^2/r_r^2) / r_r^2, finite at r = 0
 * (the reading for coincident particles: the pair then exerts no force). */
double vbco_Vr_d_over_r(double r, double E_r, double r_r)
{
    if (r >= r_r) return 0.0;
    double t = r / r_r;
    return -4.0 * E_r * (1.0 - t * t) / (r_r * r_r);
}

/* Attractive shell of eq. (softcore): -E_a (1 - u^2)^2 with
 * u = (r - (r_a + r_r)/2) / ((r_a - r_r)/2), supported on r_r < r < r_a. */
double vbco_Va(double r, double E_a, double r_r, double r_a)
{
    if (r <= r_r || r >= r_a) return 0.0;
    double m = 0.5 * (r_a + r_r);
    double w = 0.5 * (r_a - r_r);
    double u = (r - m) / w;
    double q = 1.0 - u * u;
    return -E_a * q * q;
}

/* dV_a/dr = 4 E_a u (1 - u^2) / w on the same support. */
double vbco_Va_d(double r, double E_a, double r_r, double r_a)
{
    if (r <= r_r || r >= r_a) return 0.0;
    double m = 0.5 * (r_a + r_r);
    double w = 0.5 * (r_a - r_r);
    double u = (r - m) / w;
    return 4.0 * E_a * u * (1.0 - u * u) / w;
}

/* ------------------------------------------------------------------------- */
/* Geometry                                                                   */
/* ------------------------------------------------------------------------- */

/* Minimum-image displacement x_i - x_j in a periodic box (one image per pair;
 * the box must exceed twice the largest cutoff).  Rounding of d/L is half-even. */
static void min_image(const double *xi, const double *xj, const double *L, double *d)
{
    for (int a = 0; a < 3; ++a) {
        double t = xi[a] - xj[a];
        d[a] = t - L[a] * nearbyint(t / L[a]);
    }
}

static double norm2(const double *d)
{
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* Neighbour set at radius rc: all pairs i < j whose minimum-image squared distance
 * is strictly below rc*rc, emitted in lexicographic order.  Writes at most cap pairs
 * (i, j interleaved) and returns the total number found. */
int64_t vbco_neighbor_pairs(int64_t N, const double *x, const double *L, double rc,
                            int64_t *pairs, int64_t cap)
{
    double rc2 = rc * rc;
    int64_t cnt = 0;
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = i + 1; j < N; ++j) {
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            if (norm2(d) < rc2) {
                if (cnt < cap) {
                    pairs[2 * cnt] = i;
                    pairs[2 * cnt + 1] = j;
                }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------- */
/* The corrected potential and its forces                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t N;
    const double *x;       /* N x 3 */
    const int32_t *type;   /* N, or NULL for a single type */
    const double *L;       /* 3 */
    int ntypes;
    const vbco_pair *P;    /* ntypes x ntypes, symmetric */
    const uint32_t *mask;  /* per type: bit u set => this type counts neighbours of type u */
} vbco_sys;

/* Chain exclusions (Section 6.1, where binding between stickers adjacent along one
 * strand is forbidden).  Reading: with chains of chain_len consecutive indices, two
 * particles of one chain at most excl_span beads apart neither count each other nor
 * attract; their soft-core repulsion stays.  Applies to every evaluation that follows
 * until changed; excl_span = 0 switches it off. */
static int64_t g_chain_len = 0;
static int64_t g_excl_span = 0;

void vbco_set_exclusions(int64_t chain_len, int64_t excl_span)
{
    g_chain_len = chain_len;
    g_excl_span = excl_span;
}

static int excluded(int64_t i, int64_t j)
{
    if (g_excl_span <= 0 || g_chain_len <= 1) return 0;
    if (i / g_chain_len != j / g_chain_len) return 0;
    int64_t d = i - j;
    return d <= g_excl_span && -d <= g_excl_span;
}

static int type_of(const vbco_sys *s, int64_t i) { return s->type ? s->type[i] : 0; }

static const vbco_pair *pair_of(const vbco_sys *s, int ti, int tj)
{
    return &s->P[ti * s->ntypes + tj];
}

static int counts_toward(const vbco_sys *s, int ti, int tj)
{
    if (!s->mask) return 1;
    return (int)((s->mask[ti] >> tj) & 1u);
}

/* Switching factor of one particle for one pair, eq. (Psidelta): omega(n, f - delta,
 * f - delta + 1).  With delta = 0 this is eq. (Psi).  In a multi-component system the
 * valency cap f and shift delta belong to the type pair (Section 2, multi-component
 * paragraph). */
static double switch_s(double n, const vbco_pair *p)
{
    double x1 = p->f - p->delta;
    double x2 = x1 + 1.0;
    return vbco_omega(n, x1, x2);
}

static double switch_sd(double n, const vbco_pair *p)
{
    double x1 = p->f - p->delta;
    double x2 = x1 + 1.0;
    return vbco_omega_d(n, x1, x2);
}

/* Smoothed neighbour count of particle i, eq. (counter):
 * n_i = sum over j != i of omega(r_ij, r_l, r_h), restricted to neighbour types that
 * the type of i counts, with the counting radii of the type pair. */
static double count_one(const vbco_sys *s, int64_t i)
{
    int ti = type_of(s, i);
    double n = 0.0;
    for (int64_t j = 0; j < s->N; ++j) {
        if (j == i) continue;
        int tj = type_of(s, j);
        if (!counts_toward(s, ti, tj) || excluded(i, j)) continue;
        const vbco_pair *p = pair_of(s, ti, tj);
        double d[3];
        min_image(&s->x[3 * i], &s->x[3 * j], s->L, d);
        double r = sqrt(norm2(d));
        n += vbco_omega(r, p->r_l, p->r_h);
    }
    return n;
}

/* A_i = dU/dn_i = sum_j s'_ij(n_i) s_ij(n_j) V_a,ij(r_ij): the derivative of the
 * attractive energy with respect to the count of particle i, obtained by
 * differentiating eq. (Vhat) with eq. (Psidelta) (the force expression itself is
 * in the paper's supplement, which is not available; this is its derivation). */
static double embed_one(const vbco_sys *s, const double *n, int64_t i)
{
    int ti = type_of(s, i);
    double A = 0.0;
    for (int64_t j = 0; j < s->N; ++j) {
        if (j == i || excluded(i, j)) continue;
        int tj = type_of(s, j);
        const vbco_pair *p = pair_of(s, ti, tj);
        double d[3];
        min_image(&s->x[3 * i], &s->x[3 * j], s->L, d);
        double r = sqrt(norm2(d));
        double va = vbco_Va(r, p->E_a, p->r_r, p->r_a);
        A += switch_sd(n[i], p) * switch_s(n[j], p) * va;
    }
    return A;
}

/* Pair-central scalar phi_ij = dU/dr_ij (total derivative, through the counts):
 *   V_r'(r) + Psi_ij V_a'(r) + (A_i [j counted by i] + A_j [i counted by j]) c'(r),
 * with c(r) = omega(r, r_l, r_h).  Returned divided by r; also returns the pair
 * energy V_r + Psi V_a of eq. (Vhat). */
static void pair_terms(const vbco_sys *s, const double *n, const double *A, int64_t i,
                       int64_t j, const double *d, double r2, double *phi_over_r,
                       double *epair)
{
    int ti = type_of(s, i), tj = type_of(s, j);
    const vbco_pair *p = pair_of(s, ti, tj);
    double r = sqrt(r2);
    int ex = excluded(i, j);
    double psi = ex ? 0.0 : switch_s(n[i], p) * switch_s(n[j], p);
    double e = vbco_Vr(r, p->E_r, p->r_r) + psi * vbco_Va(r, p->E_a, p->r_r, p->r_a);
    double phr = vbco_Vr_d_over_r(r, p->E_r, p->r_r);
    if (r > 0.0) {
        double dva = vbco_Va_d(r, p->E_a, p->r_r, p->r_a);
        double dc = vbco_omega_d(r, p->r_l, p->r_h);
        double chain = 0.0;
        if (counts_toward(s, ti, tj) && !ex) chain += A[i];
        if (counts_toward(s, tj, ti) && !ex) chain += A[j];
        phr += (psi * dva + chain * dc) / r;
    }
    (void)d;
    *phi_over_r = phr;
    *epair = e;
}

/* Counts n_i (eq. counter) for all particles. */
void vbco_counts(int64_t N, const double *x, const int32_t *type, const double *L,
                 int ntypes, const vbco_pair *P, const uint32_t *mask, double *n_out)
{
    vbco_sys s = {N, x, type, L, ntypes, P, mask};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) n_out[i] = count_one(&s, i);
}

/* Full evaluation.  Outputs (any may be NULL except where noted):
 *   n[N]   smoothed counts, eq. (counter)
 *   A[N]   dU/dn_i
 *   F[3N]  forces -grad U (N x 3)
 *   e[N]   per-particle energy, half of each pair energy to each partner
 *   UW[8]  U = sum_{i<j} Vhat, W = -sum_{i<j} phi_ij r_ij, and the virial tensor
 *          W_ab = -sum_{i<j} phi_ij d_a d_b / r in the order xx yy zz xy xz yz. */
void vbco_eval(int64_t N, const double *x, const int32_t *type, const double *L,
               int ntypes, const vbco_pair *P, const uint32_t *mask, double *n_out,
               double *A_out, double *F, double *e_out, double *UW)
{
    vbco_sys s = {N, x, type, L, ntypes, P, mask};
    double *n = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *A = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *rowU = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double *rowW = (double *)calloc((size_t)(N > 0 ? N : 1) * 7, sizeof(double));

    /* pass 1: counts */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) n[i] = count_one(&s, i);
    /* dU/dn */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) A[i] = embed_one(&s, n, i);
    /* forces, energies, virial */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
        double w[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            double r2 = norm2(d);
            double phr, ep;
            pair_terms(&s, n, A, i, j, d, r2, &phr, &ep);
            fx -= phr * d[0];
            fy -= phr * d[1];
            fz -= phr * d[2];
            ei += 0.5 * ep;
            if (j > i) {
                rowU[i] += ep;
                w[0] -= phr * r2;
                w[1] -= phr * d[0] * d[0];
                w[2] -= phr * d[1] * d[1];
                w[3] -= phr * d[2] * d[2];
                w[4] -= phr * d[0] * d[1];
                w[5] -= phr * d[0] * d[2];
                w[6] -= phr * d[1] * d[2];
            }
        }
        if (F) {
            F[3 * i] = fx;
            F[3 * i + 1] = fy;
            F[3 * i + 2] = fz;
        }
        if (e_out) e_out[i] = ei;
        for (int k = 0; k < 7; ++k) rowW[7 * i + k] = w[k];
    }
    if (UW) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t i = 0; i < N; ++i) {
            acc[0] += rowU[i];
            for (int k = 0; k < 7; ++k) acc[1 + k] += rowW[7 * i + k];
        }
        for (int k = 0; k < 8; ++k) UW[k] = acc[k];
    }
    if (n_out) memcpy(n_out, n, sizeof(double) * (size_t)N);
    if (A_out) memcpy(A_out, A, sizeof(double) * (size_t)N);
    free(n);
    free(A);
    free(rowU);
    free(rowW);
}

/* ------------------------------------------------------------------------- */
/* Local evaluation for large systems                                         */
/* ------------------------------------------------------------------------- */

/* Forces, counts and per-particle energies of a chosen subset of particles of a
 * large system.  The same definitions as vbco_eval, evaluated only where needed:
 * F_i depends on n and A of the particles within r_h of i, and A_j on the counts of
 * the particles within r_a of j, so counts are computed (by a full O(N) scan each)
 * only for those particles.  Every scan is over all N particles in ascending order. */
void vbco_eval_subset(int64_t N, const double *x, const int32_t *type, const double *L,
                      int ntypes, const vbco_pair *P, const uint32_t *mask,
                      const int64_t *idx, int64_t m, double *n_out, double *F_out,
                      double *e_out)
{
    vbco_sys s = {N, x, type, L, ntypes, P, mask};
    double rmax = 0.0;
    for (int k = 0; k < ntypes * ntypes; ++k) {
        if (P[k].r_r > rmax) rmax = P[k].r_r;
        if (P[k].r_a > rmax) rmax = P[k].r_a;
        if (P[k].r_h > rmax) rmax = P[k].r_h;
    }
    double rmax2 = rmax * rmax;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = idx[q];
        /* neighbours of i within the largest cutoff, ascending */
        int64_t cap = 64, nj = 0;
        int64_t *J = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            if (norm2(d) < rmax2) {
                if (nj == cap) {
                    cap *= 2;
                    J = (int64_t *)realloc(J, sizeof(int64_t) * (size_t)cap);
                }
                J[nj++] = j;
            }
        }
        /* counts of i and its neighbours; A of i and its neighbours (each A needs the
         * counts of that particle's own neighbours) */
        double *nJ = (double *)malloc(sizeof(double) * (size_t)(nj + 1));
        double *AJ = (double *)malloc(sizeof(double) * (size_t)(nj + 1));
        double n_i = count_one(&s, i);
        for (int64_t k = 0; k < nj; ++k) nJ[k] = count_one(&s, J[k]);
        for (int64_t k = -1; k < nj; ++k) {
            int64_t c = (k < 0) ? i : J[k];
            double nc = (k < 0) ? n_i : nJ[k];
            int tc = type_of(&s, c);
            double A = 0.0;
            for (int64_t j = 0; j < N; ++j) {
                if (j == c || excluded(c, j)) continue;
                int tj = type_of(&s, j);
                const vbco_pair *p = pair_of(&s, tc, tj);
                double d[3];
                min_image(&x[3 * c], &x[3 * j], L, d);
                double r2 = norm2(d);
                if (!(r2 < rmax2)) continue; /* V_a vanishes beyond r_a <= rmax */
                double r = sqrt(r2);
                double va = vbco_Va(r, p->E_a, p->r_r, p->r_a);
                if (va == 0.0) continue;
                double sd = switch_sd(nc, p);
                if (sd == 0.0) continue;
                A += sd * switch_s(count_one(&s, j), p) * va;
            }
            if (k < 0) AJ[nj] = A; else AJ[k] = A;
        }
        double fx = 0.0, fy = 0.0, fz = 0.0, ei = 0.0;
        int ti = type_of(&s, i);
        for (int64_t k = 0; k < nj; ++k) {
            int64_t j = J[k];
            int tj = type_of(&s, j);
            const vbco_pair *p = pair_of(&s, ti, tj);
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            double r2 = norm2(d);
            double r = sqrt(r2);
            int ex = excluded(i, j);
            double psi = ex ? 0.0 : switch_s(n_i, p) * switch_s(nJ[k], p);
            double ep = vbco_Vr(r, p->E_r, p->r_r) + psi * vbco_Va(r, p->E_a, p->r_r, p->r_a);
            double phr = vbco_Vr_d_over_r(r, p->E_r, p->r_r);
            if (r > 0.0) {
                double chain = 0.0;
                if (counts_toward(&s, ti, tj) && !ex) chain += AJ[nj];
                if (counts_toward(&s, tj, ti) && !ex) chain += AJ[k];
                phr += (psi * vbco_Va_d(r, p->E_a, p->r_r, p->r_a) +
                        chain * vbco_omega_d(r, p->r_l, p->r_h)) / r;
            }
            fx -= phr * d[0];
            fy -= phr * d[1];
            fz -= phr * d[2];
            ei += 0.5 * ep;
        }
        if (n_out) n_out[q] = n_i;
        if (F_out) {
            F_out[3 * q] = fx;
            F_out[3 * q + 1] = fy;
            F_out[3 * q + 2] = fz;
        }
        if (e_out) e_out[q] = ei;
        free(J);
        free(nJ);
        free(AJ);
    }
}

/* ------------------------------------------------------------------------- */
/* Harmonic bonds (bead-spring chains)                                        */
/* ------------------------------------------------------------------------- */

/* U_bond = sum over bonds of k/2 (r - r0)^2, minimum image; bonds given as index
 * pairs.  Adds the forces into F (N x 3, or NULL) and returns the bond energy.  W (7
 * doubles, or NULL) receives the bonds' virial in the convention of the pair terms,
 * W = -sum_b dU_b/dr r and W_ab = -sum_b dU_b/dr d_a d_b / r, with dU_b/dr = k (r - r0),
 * ordered {W, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz}. */
double vbco_bonds(int64_t N, const double *x, const double *L, const int64_t *bonds,
                  int64_t nb, double k, double r0, double *F, double *W)
{
    (void)N;
    double U = 0.0;
    double w[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < nb; ++b) {
        int64_t i = bonds[2 * b], j = bonds[2 * b + 1];
        double d[3];
        min_image(&x[3 * i], &x[3 * j], L, d);
        double r = sqrt(norm2(d));
        double dr = r - r0;
        U += 0.5 * k * dr * dr;
        double c = r > 0.0 ? k * dr / r : 0.0; /* dU_b/dr / r */
        if (F && r > 0.0) {
            for (int a = 0; a < 3; ++a) {
                F[3 * i + a] -= c * d[a];
                F[3 * j + a] += c * d[a];
            }
        }
        w[0] -= c * (r * r);
        w[1] -= c * d[0] * d[0];
        w[2] -= c * d[1] * d[1];
        w[3] -= c * d[2] * d[2];
        w[4] -= c * d[0] * d[1];
        w[5] -= c * d[0] * d[2];
        w[6] -= c * d[1] * d[2];
    }
    if (W)
        for (int a = 0; a < 7; ++a) W[a] = w[a];
    return U;
}

/* ------------------------------------------------------------------------- */
/* Observables of valency control                                             */
/* ------------------------------------------------------------------------- */

/* Section 3: two particles count as neighbours when their separation is below the
 * attraction range, r_ij < r_a (an instantaneous criterion); z_i is the number of such
 * neighbours of i.  The penetration count p_i of the stability study (Section 6.2) is the
 * number of particles within the repulsive core, r_ij < r_r.  Both use the radii of the
 * pair (type_i, type_j) and decide r^2 < r * r in FP64 on the minimum image. */
void vbco_observables(int64_t N, const double *x, const int32_t *type, const double *L,
                      int ntypes, const vbco_pair *P, int32_t *z, int32_t *pen)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int ti = type ? type[i] : 0;
        int32_t zi = 0, pi = 0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            int tj = type ? type[j] : 0;
            const vbco_pair *p = &P[ti * ntypes + tj];
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            double r2 = norm2(d);
            if (r2 < p->r_a * p->r_a) ++zi;
            if (r2 < p->r_r * p->r_r) ++pi;
        }
        z[i] = zi;
        pen[i] = pi;
    }
}

/* Clusters of the bond graph (Section 3): i and j are bonded when r_ij < r_a of the pair
 * (type_i, type_j), the neighbour criterion of z_i above; clusters are the connected
 * components.  Plain union-find over all pairs i < j, in index order, linking the root with
 * the larger index under the one with the smaller, so that every particle ends with the
 * smallest index of its cluster as its label.  z_i (bonds of i) is returned alongside. */
static int64_t uf_find(int64_t *parent, int64_t a)
{
    while (parent[a] != a) a = parent[a];
    return a;
}

void vbco_bond_clusters(int64_t N, const double *x, const int32_t *type, const double *L, int ntypes,
                        const vbco_pair *P, int64_t *label, int32_t *z)
{
    for (int64_t i = 0; i < N; ++i) {
        label[i] = i;
        z[i] = 0;
    }
    for (int64_t i = 0; i < N; ++i) {
        int ti = type ? type[i] : 0;
        for (int64_t j = i + 1; j < N; ++j) {
            int tj = type ? type[j] : 0;
            const vbco_pair *p = &P[ti * ntypes + tj];
            double d[3];
            min_image(&x[3 * i], &x[3 * j], L, d);
            if (!(norm2(d) < p->r_a * p->r_a)) continue;
            ++z[i];
            ++z[j];
            int64_t a = uf_find(label, i), b = uf_find(label, j);
            if (a < b) label[b] = a;
            else if (b < a) label[a] = b;
        }
    }
    for (int64_t i = 0; i < N; ++i) label[i] = uf_find(label, i);
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: Philox4x32-10                                */
/* ------------------------------------------------------------------------- */

/* Philox4x32 with 10 rounds, from its published definition (Salmon, Moraes, Dror &
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): each round multiplies
 * counter words 0 and 2 by two fixed odd 32-bit constants, takes the high and low halves
 * of the 64-bit products, mixes the high halves with the other counter words and the
 * round key, and bumps the key by two Weyl constants between rounds. */
void vbco_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Langevin noise of one particle for one step.  Reading (the paper states only the
 * friction): key = the two 32-bit halves of seed (low first), counter = the halves of
 * step, then of tag; each of the first three output words w gives a uniform
 * u = (w + 1/2) 2^-32 in (0, 1), turned into a zero-mean, unit-variance variate
 * sqrt(3) (2u - 1).  Only exactly rounded operations are used, so any other
 * implementation of the same steps reproduces it bit for bit. */
void vbco_noise(uint64_t seed, uint64_t tag, uint64_t step, double xi[3])
{
    const double SQRT3 = 1.7320508075688772;
    uint32_t ctr[4] = {(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)tag, (uint32_t)(tag >> 32)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    vbco_philox4x32_10(ctr, key, w);
    for (int a = 0; a < 3; ++a) {
        double u = ((double)w[a] + 0.5) * 0x1.0p-32;
        xi[a] = (2.0 * u - 1.0) * SQRT3;
    }
}

/* ------------------------------------------------------------------------- */
/* Time integration                                                           */
/* ------------------------------------------------------------------------- */

static void wrap_all(int64_t N, double *x, const double *L)
{
    for (int64_t i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) {
            double t = x[3 * i + a];
            if (t >= L[a]) t -= L[a];
            else if (t < 0.0) t += L[a];
            x[3 * i + a] = t;
        }
}

static void total_force(const vbco_sys *s, const int64_t *bonds, int64_t nb, double kb,
                        double r0, double *F, double *U)
{
    double UW[8];
    vbco_eval(s->N, s->x, s->type, s->L, s->ntypes, s->P, s->mask, NULL, NULL, F, NULL, UW);
    double Ub = 0.0;
    if (bonds && nb > 0) Ub = vbco_bonds(s->N, s->x, s->L, bonds, nb, kb, r0, F, NULL);
    if (U) *U = UW[0] + Ub;
}

/* Integrate nsteps steps in place (x, v: N x 3; unit masses).
 *   kind 0: velocity Verlet   v += dt/2 F; x += dt v; wrap; F = F(x); v += dt/2 F
 *   kind 1: Langevin BAOAB     v += dt/2 F; x += dt/2 v; v = c1 v + c2s xi;
 *                              x += dt/2 v; wrap; F = F(x); v += dt/2 F
 * with c1 = exp(-gamma dt), c2s = sqrt(1 - c1^2) sqrt(kT) and xi from vbco_noise keyed
 * by (seed, tag[i]) at counter step0 + k for step k.  (BAOAB is the reading for the
 * paper's Langevin thermostat with friction gamma.)  Optional outputs: F (final
 * forces), U_hist / K_hist (potential and kinetic energy after every step). */
void vbco_run(int64_t N, double *x, double *v, const int32_t *type, const int64_t *tag,
              const double *L, int ntypes, const vbco_pair *P, const uint32_t *mask,
              const int64_t *bonds, int64_t nb, double kb, double r0, int kind, double dt,
              double kT, double gamma, uint64_t seed, uint64_t step0, int64_t nsteps,
              double *F_out, double *U_hist, double *K_hist)
{
    vbco_sys s = {N, x, type, L, ntypes, P, mask};
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1));
    double c1 = exp(-gamma * dt);
    double c2s = sqrt(1.0 - c1 * c1) * sqrt(kT);
    double hdt = 0.5 * dt;
    total_force(&s, bonds, nb, kb, r0, F, NULL);
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int64_t i = 0; i < 3 * N; ++i) v[i] += hdt * F[i];
        if (kind == 0) {
            for (int64_t i = 0; i < 3 * N; ++i) x[i] += dt * v[i];
        } else {
            for (int64_t i = 0; i < 3 * N; ++i) x[i] += hdt * v[i];
            for (int64_t i = 0; i < N; ++i) {
                double xi[3];
                vbco_noise(seed, (uint64_t)(tag ? tag[i] : i), step0 + (uint64_t)k, xi);
                for (int a = 0; a < 3; ++a) v[3 * i + a] = c1 * v[3 * i + a] + c2s * xi[a];
            }
            for (int64_t i = 0; i < 3 * N; ++i) x[i] += hdt * v[i];
        }
        wrap_all(N, x, L);
        double U = 0.0;
        total_force(&s, bonds, nb, kb, r0, F, &U);
        for (int64_t i = 0; i < 3 * N; ++i) v[i] += hdt * F[i];
        if (U_hist) U_hist[k] = U;
        if (K_hist) {
            double K = 0.0;
            for (int64_t i = 0; i < 3 * N; ++i) K += 0.5 * v[i] * v[i];
            K_hist[k] = K;
        }
    }
    if (F_out) memcpy(F_out, F, sizeof(double) * 3 * (size_t)N);
    free(F);
}
