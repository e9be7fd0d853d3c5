/*
 * h4d_oracle.c -- plain FP64 CPU reference of the H4D ion-pair exchange
 * (Kim, Belloni & Rotenberg, arXiv 2307.11447).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.  It
 * shares no code with the GPU path.  Slow on purpose: every energy or force
 * evaluation re-enumerates the pairs, all sums run left to right in FP64.
 *
 * Timing build.  Compiled with -fopenmp (liboracle_omp.so, for the
 * benchmark's CPU baseline only), the pair enumeration and the pair sum of
 * every energy or force evaluation, and the candidate features of the
 * learned proposal, spread over threads; the pair order is the serial one,
 * but the energy and force sums are reduced per thread, so that build
 * rounds differently.  The parity build has no -fopenmp: the pragmas are
 * ignored and every sum runs in the order written.
 *
 * Physics (one pair i<j, minimum image r_ij):
 *   s^2 = |r_ij|^2 + (w_i - w_j)^2, w = altitude of a flyer, 0 otherwise
 *     (the 4D distance of Sec. I and Sec. II C);
 *   truncated and shifted Lennard-Jones, Eq. (19), force not shifted,
 *     Lorentz-Berthelot mixing (Sec. II D 2);
 *   damped shifted force Coulomb (Fennell & Gezelter 2006), the
 *     Wolf-family real-space-only electrostatics mentioned in Sec. II B 2,
 *     multiplied by g = exp(-kappa_sr * w) when exactly one of i, j is
 *     flying (short-range screening, Eq. 11);
 *   intramolecular pairs of a rigid water are excluded.
 */
#include "h4d_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x64-10 from its published definition (Salmon, Moraes, Dror & */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).        */
/* ------------------------------------------------------------------ */
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        __uint128_t p0 = (__uint128_t)M0 * x0;
        __uint128_t p1 = (__uint128_t)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The top 52 random bits -> uniform in the open interval (0, 1): the
 * midpoints (m + 1/2) 2^-52 are exact doubles, the largest is 1 - 2^-53. */
double or_u01(uint64_t bits)
{
    return ((double)(bits >> 12) + 0.5) * 0x1p-52;
}

static int trial_begin(const or_params *p, or_state *s, uint64_t trial, int force_move,
                       const or_proposal *prop, or_trial_rec *rec, int *ic_out, int *ia_out, int *nf_out,
                       double *feat_out);

static void draw4(const or_params *p, uint64_t a, uint64_t b, uint64_t c, double u[4])
{
    uint64_t ctr[4] = {a, b, c, 0}, key[2] = {p->seed, p->stream}, o[4];
    or_philox4x64(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = or_u01(o[i]);
}

/* Counter purposes: move and plain sites, Maxwell-Boltzmann momenta, N_f,
 * candidate sites of the learned proposal, its categorical choice. */
enum { PURPOSE_SELECT = 1, PURPOSE_MB = 2, PURPOSE_NSTEPS = 3, PURPOSE_CAND = 4, PURPOSE_PICK = 5,
       PURPOSE_BIAS = 6, PURPOSE_REVERSE = 7, PURPOSE_MD = 8, PURPOSE_REFRESH = 9, PURPOSE_INITV = 10 };

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */
/* Periodic wrap into [0, L).  Coordinates are never more than one edge
 * outside the box, so one shift is exact; the floor form is kept for the
 * general case. */
static double wrap1(double x, double L)
{
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
    if (x >= 0.0 && x < L) return x;
    double y = x - L * floor(x / L);
    return (y >= L || y < 0.0) ? 0.0 : y;
}

static double minimg(double d, double L)
{
    return d - L * nearbyint(d / L);
}

/* ------------------------------------------------------------------ */
/* Pair potential                                                      */
/* ------------------------------------------------------------------ */
int or_pair(const or_params *p, int ti, int tj, double s2, double g,
            double *u_lj, double *u_c, double *dlj_ds, double *dc_ds)
{
    *u_lj = 0.0; *u_c = 0.0; *dlj_ds = 0.0; *dc_ds = 0.0;
    if (ti < 0 || tj < 0 || ti >= p->n_types || tj >= p->n_types) return -1;
    const double s = sqrt(s2);
    /* Eq. (19): truncated and shifted LJ, Lorentz-Berthelot mixing. */
    const double sig = 0.5 * (p->sigma[ti] + p->sigma[tj]);
    const double eps = sqrt(p->eps[ti] * p->eps[tj]);
    if (eps > 0.0 && s < p->rc_lj) {
        const double a = pow(sig / s, 6.0);
        const double ac = pow(sig / p->rc_lj, 6.0);
        *u_lj = 4.0 * eps * (a * a - a - ac * ac + ac);
        *dlj_ds = 4.0 * eps * (-12.0 * a * a + 6.0 * a) / s;
    }
    /* Damped shifted force Coulomb. */
    const double qq = p->charge[ti] * p->charge[tj];
    if (qq != 0.0 && s < p->rc_coul) {
        const double al = p->alpha, Rc = p->rc_coul;
        const double erfc_c = erfc(al * Rc);
        const double Sc = erfc_c / (Rc * Rc) + 2.0 * al / sqrt(M_PI) * exp(-al * al * Rc * Rc) / Rc;
        const double u = p->ke * qq * (erfc(al * s) / s - erfc_c / Rc + Sc * (s - Rc));
        const double du = p->ke * qq * (-erfc(al * s) / (s * s)
                                        - 2.0 * al / sqrt(M_PI) * exp(-al * al * s * s) / s + Sc);
        *u_c = g * u;
        *dc_ds = g * du;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Pair enumeration: all pairs i<j with 3D minimum-image r < rcut      */
/* (a superset of the pairs within the 4D cutoff, since s >= r).       */
/* ------------------------------------------------------------------ */
typedef struct { int32_t *i, *j; int64_t n, cap; } pairlist;

static int pl_push(pairlist *pl, int i, int j)
{
    if (pl->n == pl->cap) {
        int64_t nc = pl->cap ? 2 * pl->cap : 4096;
        int32_t *ni = realloc(pl->i, nc * sizeof(int32_t));
        if (!ni) return -1;
        pl->i = ni;
        int32_t *nj = realloc(pl->j, nc * sizeof(int32_t));
        if (!nj) return -1;
        pl->j = nj;
        pl->cap = nc;
    }
    pl->i[pl->n] = i; pl->j[pl->n] = j; pl->n++;
    return 0;
}

static void pl_free(pairlist *pl) { free(pl->i); free(pl->j); }

static int excluded(const or_state *s, int i, int j)
{
    return s->mol[i] >= 0 && s->mol[i] == s->mol[j];
}

static double r2_of(const or_params *p, const or_state *s, int i, int j)
{
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double dd = minimg(s->x[3 * i + d] - s->x[3 * j + d], p->box[d]);
        r2 += dd * dd;
    }
    return r2;
}

/* The pairs (i, j > i) of atom i from the 27 cells around its own. */
static int cell_pairs(const or_params *p, const or_state *s, int i, const int nc[3], const int *head,
                      const int *next, const int *cid, double rc2, pairlist *pl)
{
    int c = cid[i];
    int cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int ax = (cx + dx + nc[0]) % nc[0];
                int ay = (cy + dy + nc[1]) % nc[1];
                int az = (cz + dz + nc[2]) % nc[2];
                int cc = (az * nc[1] + ay) * nc[0] + ax;
                for (int j = head[cc]; j >= 0; j = next[j])
                    if (j > i && !excluded(s, i, j) && r2_of(p, s, i, j) < rc2)
                        if (pl_push(pl, i, j)) return -1;
            }
    return 0;
}

static int enumerate_pairs(const or_params *p, const or_state *s, double rcut, pairlist *pl)
{
    const int n = s->n;
    const double rc2 = rcut * rcut;
    int nc[3];
    int cells = p->use_cells;
    for (int d = 0; d < 3; ++d) {
        nc[d] = (int)floor(p->box[d] / rcut);
        if (nc[d] < 3) cells = 0;
    }
    if (!cells) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                if (!excluded(s, i, j) && r2_of(p, s, i, j) < rc2)
                    if (pl_push(pl, i, j)) return -1;
        return 0;
    }
    /* Linked cells (Allen & Tildesley): head/next lists, 27-cell stencil. */
    const int ncell = nc[0] * nc[1] * nc[2];
    int *head = malloc(ncell * sizeof(int));
    int *next = malloc((n > 0 ? n : 1) * sizeof(int));
    int *cid = malloc((n > 0 ? n : 1) * sizeof(int));
    if (!head || !next || !cid) { free(head); free(next); free(cid); return -1; }
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int c3[3];
        for (int d = 0; d < 3; ++d) {
            int k = (int)floor(s->x[3 * i + d] / p->box[d] * nc[d]);
            if (k < 0) k = 0;
            if (k >= nc[d]) k = nc[d] - 1;
            c3[d] = k;
        }
        int c = (c3[2] * nc[1] + c3[1]) * nc[0] + c3[0];
        cid[i] = c;
        next[i] = head[c];
        head[c] = i;
    }
    int err = 0;
#ifdef _OPENMP
    /* timing build: each thread lists the pairs of a contiguous range of i,
     * and the lists are joined in thread order, i.e. in the serial order */
    int nt = omp_get_max_threads();
    pairlist *part = calloc((size_t)nt, sizeof(pairlist));
    if (!part) { free(head); free(next); free(cid); return -1; }
#pragma omp parallel num_threads(nt) reduction(|:err)
    {
        const int t = omp_get_thread_num();
        const int lo = (int)((int64_t)n * t / nt), hi = (int)((int64_t)n * (t + 1) / nt);
        for (int i = lo; i < hi && !err; ++i) err |= cell_pairs(p, s, i, nc, head, next, cid, rc2, &part[t]);
    }
    for (int t = 0; t < nt; ++t) {
        for (int64_t q = 0; q < part[t].n && !err; ++q) err |= pl_push(pl, part[t].i[q], part[t].j[q]);
        pl_free(&part[t]);
    }
    free(part);
#else
    for (int i = 0; i < n && !err; ++i) err |= cell_pairs(p, s, i, nc, head, next, cid, rc2, pl);
#endif
    free(head); free(next); free(cid);
    return err ? -1 : 0;
}

/* Pairs that involve a flyer: flyer x every other atom, flyer-flyer once. */
static int enumerate_fly_pairs(const or_params *p, const or_state *s, double rcut, pairlist *pl)
{
    const double rc2 = rcut * rcut;
    for (int i = 0; i < s->n; ++i) {
        if (!s->flying[i]) continue;
        for (int j = 0; j < s->n; ++j) {
            if (j == i) continue;
            if (s->flying[j] && j < i) continue;
            if (!excluded(s, i, j) && r2_of(p, s, i, j) < rc2)
                if (pl_push(pl, i < j ? i : j, i < j ? j : i)) return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Energy and forces                                                   */
/* ------------------------------------------------------------------ */
/* Species-specific w_max (supplement): both flyers reach w = 0 together,
 * the anion's altitude r_w times the cation's all along the schedule, so
 * w is the cation's altitude and each flyer has its own factor. */
static double w_ratio(const or_params *p) { return p->w_max_ratio > 0.0 ? p->w_max_ratio : 1.0; }

static double flyer_factor(const or_params *p, int type) { return type == p->anion_type ? w_ratio(p) : 1.0; }

int or_compute(const or_params *p, const or_state *s, double w, int mode,
               double *F, or_energy *e)
{
    memset(e, 0, sizeof(*e));
    if (F) memset(F, 0, 3 * (size_t)s->n * sizeof(double));
    const double rcut = p->rc_lj > p->rc_coul ? p->rc_lj : p->rc_coul;
    /* minimum image is the whole periodic sum only if every edge >= 2 r_cut */
    for (int d = 0; d < 3; ++d)
        if (p->box[d] < 2.0 * rcut) return -7;
    pairlist pl = {0};
    int rc = (mode == OR_MODE_FLY) ? enumerate_fly_pairs(p, s, rcut, &pl)
                                   : enumerate_pairs(p, s, rcut, &pl);
    if (rc) { pl_free(&pl); return -1; }
    /* Eq. 11 screening at the flyers' mean altitude (Sec. II B 2: with
     * several flyers at different altitudes, the average one) */
    const double wbar = 0.5 * w * (1.0 + w_ratio(p));
    const double gscr = exp(-p->kappa_sr * wbar);
    double U = 0.0, U_lj = 0.0, U_c = 0.0, virial = 0.0, dUdw = 0.0;
#ifdef _OPENMP
    /* timing build: per-thread force copies, summed at the end */
    const int nf3 = 3 * s->n;
    double *Fsum = F ? F : calloc((size_t)nf3 + 1, sizeof(double));
    if (!Fsum) { pl_free(&pl); return -1; }
#pragma omp parallel for schedule(static) reduction(+:U, U_lj, U_c, virial, dUdw) reduction(+:Fsum[:nf3])
#else
    double *Fsum = F;
#endif
    for (int64_t k = 0; k < pl.n; ++k) {
        const int i = pl.i[k], j = pl.j[k];
        const int fi = s->flying[i], fj = s->flying[j];
        if (mode == OR_MODE_EXCL && (fi || fj)) continue;
        if (mode == OR_MODE_FLY && !(fi || fj)) continue;
        double r[3], r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            r[d] = minimg(s->x[3 * i + d] - s->x[3 * j + d], p->box[d]);
            r2 += r[d] * r[d];
        }
        const double ri = fi ? flyer_factor(p, s->type[i]) : 0.0, rj = fj ? flyer_factor(p, s->type[j]) : 0.0;
        const double wi = ri * w, wj = rj * w;
        const double dw = wi - wj;
        const double s2 = r2 + dw * dw;
        const int one_flying = (fi != fj);
        const double g = one_flying ? gscr : 1.0;
        double ulj, uc, dlj, dc;
        or_pair(p, s->type[i], s->type[j], s2, g, &ulj, &uc, &dlj, &dc);
        const double sd = sqrt(s2);
        const double duds = dlj + dc;
        U_lj += ulj;
        U_c += uc;
        U += ulj + uc;
        /* F_i = -du/ds * (r_i - r_j)/s, virial sum r_ij . F_ij (3D part). */
        const double fs = -duds / sd;
        virial += fs * r2;
        if (Fsum) {
            for (int d = 0; d < 3; ++d) {
                Fsum[3 * i + d] += fs * r[d];
                Fsum[3 * j + d] -= fs * r[d];
            }
        }
        /* dU/dw: ds/dw = dw (r_i - r_j) / s with the flyers' factors r;
         * dg/dw = -kappa_sr (1 + r_w) / 2 g for a flyer-nonflyer pair. */
        if (sd > 0.0) dUdw += duds * (dw * (ri - rj) / sd);
        if (one_flying) dUdw -= p->kappa_sr * 0.5 * (1.0 + w_ratio(p)) * uc;
    }
#ifdef _OPENMP
    if (!F) free(Fsum);
#endif
    e->U = U; e->U_lj = U_lj; e->U_c = U_c; e->virial = virial; e->dUdw = dUdw;
    pl_free(&pl);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Momenta                                                             */
/* ------------------------------------------------------------------ */
/* A Maxwell-Boltzmann velocity of atom i: each 3D component ~ N(0, kT/m)
 * (Sec. II A), normals from the Box-Muller transform of two uniforms of the
 * stream (counter, purpose, tag). */
static void mb_velocity(const or_params *p, const or_state *s, int i, uint64_t counter, uint64_t purpose,
                        double out[3])
{
    double u[4];
    draw4(p, counter, purpose, (uint64_t)s->tag[i], u);
    const double r01 = sqrt(-2.0 * log(u[0]));
    const double r23 = sqrt(-2.0 * log(u[2]));
    const double sd = sqrt(p->accel * p->kT / p->mass[s->type[i]]);
    out[0] = sd * r01 * cos(2.0 * M_PI * u[1]);
    out[1] = sd * r01 * sin(2.0 * M_PI * u[1]);
    out[2] = sd * r23 * cos(2.0 * M_PI * u[3]);
}

int or_mb_velocities(const or_params *p, or_state *s, uint64_t trial)
{
    for (int i = 0; i < s->n; ++i) mb_velocity(p, s, i, trial, PURPOSE_MB, s->v + 3 * i);
    if (p->water) return or_constrain_velocities(p, s);
    return 0;
}

int or_init_velocities(const or_params *p, or_state *s)
{
    for (int i = 0; i < s->n; ++i) mb_velocity(p, s, i, 0, PURPOSE_INITV, s->v + 3 * i);
    /* rigid waters: Maxwell-Boltzmann momenta restricted to the constraint
     * surface (the velocity constraint removes the bond components) */
    if (p->water) return or_constrain_velocities(p, s);
    return 0;
}

/* Signs of the symmetric two-end momentum reversal of a trial: each end
 * reverses every momentum with probability 1/2. */
static void reversal_signs(const or_params *p, uint64_t trial, double *s0, double *s1)
{
    double u[4];
    draw4(p, trial, PURPOSE_REVERSE, 0, u);
    *s0 = u[0] < 0.5 ? -1.0 : 1.0;
    *s1 = u[1] < 0.5 ? -1.0 : 1.0;
}

double or_kinetic(const or_params *p, const or_state *s)
{
    double K = 0.0;
    for (int i = 0; i < s->n; ++i) {
        if (s->flying[i]) continue;
        const double m = p->mass[s->type[i]];
        for (int d = 0; d < 3; ++d) K += 0.5 * m * s->v[3 * i + d] * s->v[3 * i + d] / p->accel;
    }
    return K;
}

/* ------------------------------------------------------------------ */
/* Rigid water: the three distance constraints O-H1, O-H2, H1-H2.      */
/* Positions: iterate the bond-by-bond correction along the reference  */
/* bond vectors until every constraint holds to 1e-14 relative (the    */
/* constraint problem that an analytic solver also solves).            */
/* ------------------------------------------------------------------ */
static void bond_list(const or_params *p, int m, int a[3], int b[3], double d[3])
{
    const int o = 3 * m;
    a[0] = o; b[0] = o + 1; d[0] = p->d_oh;
    a[1] = o; b[1] = o + 2; d[1] = p->d_oh;
    a[2] = o + 1; b[2] = o + 2; d[2] = p->d_hh;
}

int or_constrain_positions(const or_params *p, or_state *s, const double *xref)
{
    for (int m = 0; m < s->n_mol; ++m) {
        int a[3], b[3];
        double d[3], corr[9] = {0};
        bond_list(p, m, a, b, d);
        /* local unwrapped copy relative to the oxygen: O(1) magnitudes keep
         * the rounding of |s|^2 far below the convergence tolerance */
        double xl[9];
        const int o = 3 * m;
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c)
                xl[3 * k + c] = k ? minimg(s->x[3 * (o + k) + c] - s->x[3 * o + c], p->box[c]) : 0.0;
        int it;
        for (it = 0; it < 1000; ++it) {
            int done = 1;
            for (int q = 0; q < 3; ++q) {
                const int la = a[q] - o, lb = b[q] - o;
                double sv[3], rr[3], ss = 0.0, sr = 0.0;
                for (int c = 0; c < 3; ++c) {
                    sv[c] = xl[3 * la + c] - xl[3 * lb + c];
                    rr[c] = minimg(xref[3 * a[q] + c] - xref[3 * b[q] + c], p->box[c]);
                    ss += sv[c] * sv[c];
                    sr += sv[c] * rr[c];
                }
                const double diff = d[q] * d[q] - ss;
                if (fabs(diff) > 1e-13 * d[q] * d[q]) done = 0;
                const double ima = 1.0 / p->mass[s->type[a[q]]], imb = 1.0 / p->mass[s->type[b[q]]];
                const double gq = diff / (2.0 * sr * (ima + imb));
                for (int c = 0; c < 3; ++c) {
                    xl[3 * la + c] += gq * rr[c] * ima;
                    xl[3 * lb + c] -= gq * rr[c] * imb;
                    corr[3 * la + c] += gq * rr[c] * ima;
                    corr[3 * lb + c] -= gq * rr[c] * imb;
                }
            }
            if (done) break;
        }
        if (it == 1000) return -2;
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                const int i = o + k;
                s->x[3 * i + c] = wrap1(s->x[3 * i + c] + corr[3 * k + c], p->box[c]);
                s->v[3 * i + c] += corr[3 * k + c] / p->dt;
            }
    }
    return 0;
}

/* Velocities: find the three multipliers that make every bond's relative
 * velocity orthogonal to the bond (a 3x3 linear system, Gaussian
 * elimination with partial pivoting). */
int or_constrain_velocities(const or_params *p, or_state *s)
{
    for (int m = 0; m < s->n_mol; ++m) {
        int a[3], b[3];
        double d[3], r[3][3], A[3][4];
        bond_list(p, m, a, b, d);
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c)
                r[q][c] = minimg(s->x[3 * a[q] + c] - s->x[3 * b[q] + c], p->box[c]);
        for (int k = 0; k < 3; ++k) {
            /* row k: (v_a' - v_b') . r_k = 0, v_x' = v_x + sum_l lam_l c_{x,l} r_l / m_x */
            const int pk = a[k], qk = b[k];
            const double ip = 1.0 / p->mass[s->type[pk]], iq = 1.0 / p->mass[s->type[qk]];
            for (int l = 0; l < 3; ++l) {
                const double cp = (pk == a[l]) ? 1.0 : (pk == b[l] ? -1.0 : 0.0);
                const double cq = (qk == a[l]) ? 1.0 : (qk == b[l] ? -1.0 : 0.0);
                double dot = 0.0;
                for (int c = 0; c < 3; ++c) dot += r[l][c] * r[k][c];
                A[k][l] = dot * (cp * ip - cq * iq);
            }
            double rhs = 0.0;
            for (int c = 0; c < 3; ++c) rhs -= (s->v[3 * pk + c] - s->v[3 * qk + c]) * r[k][c];
            A[k][3] = rhs;
        }
        for (int col = 0; col < 3; ++col) {
            int piv = col;
            for (int rr = col + 1; rr < 3; ++rr)
                if (fabs(A[rr][col]) > fabs(A[piv][col])) piv = rr;
            if (A[piv][col] == 0.0) return -2;
            if (piv != col)
                for (int c = 0; c < 4; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
            for (int rr = 0; rr < 3; ++rr) {
                if (rr == col) continue;
                const double f = A[rr][col] / A[col][col];
                for (int c = col; c < 4; ++c) A[rr][c] -= f * A[col][c];
            }
        }
        double lam[3];
        for (int q = 0; q < 3; ++q) lam[q] = A[q][3] / A[q][q];
        for (int l = 0; l < 3; ++l) {
            const double ia = 1.0 / p->mass[s->type[a[l]]], ib = 1.0 / p->mass[s->type[b[l]]];
            for (int c = 0; c < 3; ++c) {
                s->v[3 * a[l] + c] += lam[l] * r[l][c] * ia;
                s->v[3 * b[l] + c] -= lam[l] * r[l][c] * ib;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* NEMD                                                                */
/* ------------------------------------------------------------------ */
double or_altitude(const or_params *p, int move, int k, int nf)
{
    /* Eq. (2), constant vertical velocity: insertion from w_max down to 0,
     * deletion from 0 up to w_max.  The supplement's variable-velocity
     * schedules, with x the insertion's reduced time k / nf:
     * w_max (1 - x^n) and w_max (1 - x)^n.  A deletion runs the insertion's
     * schedule backwards in time (x = (nf - k) / nf), the reverse path that
     * detailed balance pairs with it. */
    if (nf <= 0) return 0.0;   /* an instantaneous exchange switches at once */
    const int j = move > 0 ? k : nf - k;
    if (p->schedule == 1) return p->w_max * (1.0 - pow((double)j / (double)nf, p->schedule_n));
    if (p->schedule == 2) return p->w_max * pow(1.0 - (double)j / (double)nf, p->schedule_n);
    if (move > 0) return p->w_max * (double)(nf - k) / (double)nf;
    return p->w_max * (double)k / (double)nf;
}

static double u_fly(const or_params *p, const or_state *s, double w)
{
    or_energy e;
    if (or_compute(p, s, w, OR_MODE_FLY, NULL, &e)) return NAN;
    return e.U;
}

int or_nemd(const or_params *p, or_state *s, int move, int nf, double *W)
{
    const int n = s->n;
    double *F = malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double *xref = p->water ? malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double)) : NULL;
    if (!F || (p->water && !xref)) { free(F); free(xref); return -1; }
    or_energy e;
    double Wp = 0.0;
    int rc = 0;
    if (or_compute(p, s, or_altitude(p, move, 0, nf), OR_MODE_NEMD, F, &e)) {
        free(F); free(xref); return -7;
    }
    for (int k = 0; k < nf; ++k) {
        const double h = 0.5 * p->dt;
        const double dU_start = u_fly(p, s, or_altitude(p, move, k + 1, nf)) -
                                u_fly(p, s, or_altitude(p, move, k, nf));
        /* half kick with F(x_k; w_k), then drift; flyers stay fixed in 3D */
        for (int i = 0; i < n; ++i) {
            if (s->flying[i]) continue;
            const double m = p->mass[s->type[i]];
            for (int d = 0; d < 3; ++d) s->v[3 * i + d] += h * p->accel * F[3 * i + d] / m;
        }
        if (xref) memcpy(xref, s->x, 3 * (size_t)n * sizeof(double));
        for (int i = 0; i < n; ++i) {
            if (s->flying[i]) continue;
            for (int d = 0; d < 3; ++d)
                s->x[3 * i + d] = wrap1(s->x[3 * i + d] + p->dt * s->v[3 * i + d], p->box[d]);
        }
        if (xref && (rc = or_constrain_positions(p, s, xref))) break;
        /* protocol work of the step: the altitude increment w_k -> w_{k+1}
         * of U_fly, averaged over the two ends x_k and x_{k+1} (trapezoid,
         * the quadrature that matches the symmetric kick-drift-kick) */
        const double wk = or_altitude(p, move, k, nf), wk1 = or_altitude(p, move, k + 1, nf);
        Wp += 0.5 * (dU_start + (u_fly(p, s, wk1) - u_fly(p, s, wk)));
        /* second half kick with F(x_{k+1}; w_{k+1}) */
        or_compute(p, s, wk1, OR_MODE_NEMD, F, &e);
        for (int i = 0; i < n; ++i) {
            if (s->flying[i]) continue;
            const double m = p->mass[s->type[i]];
            for (int d = 0; d < 3; ++d) s->v[3 * i + d] += h * p->accel * F[3 * i + d] / m;
        }
        if (p->water && (rc = or_constrain_velocities(p, s))) break;
    }
    free(F); free(xref);
    *W = Wp;
    return rc;
}

/* ------------------------------------------------------------------ */
/* One grand-canonical trial                                           */
/* ------------------------------------------------------------------ */
/* ------------------------------------------------------------------ */
/* Bimodal bias of the flying anion's position given the cation's       */
/* (Sec. II B 4, Eqs. 12-16).                                           */
/* ------------------------------------------------------------------ */
double or_bias_b(double x, double L, double xb, double alpha)
{
    /* Eq. (14): two Gaussians at +-x_b, normalised on [-L/2, L/2] */
    const double sa = sqrt(alpha);
    const double num = exp(-alpha * (x - xb) * (x - xb)) + exp(-alpha * (x + xb) * (x + xb));
    const double den = erf(sa * (xb + 0.5 * L)) - erf(sa * (xb - 0.5 * L));
    return sqrt(alpha / M_PI) * num / den;
}

double or_bias_B(const or_params *p, const double xa[3], const double xc[3])
{
    /* Eq. (12): V times the product of the three one-dimensional densities */
    double B = p->box[0] * p->box[1] * p->box[2];
    for (int d = 0; d < 3; ++d) {
        const double L = p->box[d];
        double x = xa[d] - xc[d];
        x -= L * round(x / L);
        B *= or_bias_b(x, L, p->bias_xb, p->bias_alpha);
    }
    return B;
}

double or_bias_offset(const or_params *p, uint64_t trial, int d)
{
    /* one uniform picks the Gaussian at -x_b or +x_b (equal masses on the
     * symmetric edge), Box-Muller draws from it, and a draw outside
     * [-L/2, L/2] is replaced by the next attempt's: a draw from Eq. (14) */
    const double L = p->box[d];
    for (int attempt = 0; attempt < 64; ++attempt) {
        double u[4];
        draw4(p, trial, PURPOSE_BIAS, (uint64_t)(4 * attempt + d), u);
        const double mu = u[0] < 0.5 ? -p->bias_xb : p->bias_xb;
        const double z = sqrt(-2.0 * log(u[1])) * cos(6.283185307179586476925286766559 * u[2]);
        const double x = mu + z / sqrt(2.0 * p->bias_alpha);
        if (fabs(x) <= 0.5 * L) return x;
    }
    return NAN;
}

/* anion indices in ascending tag order */
static int anions_by_tag(const or_params *p, const or_state *s, int *idx)
{
    int m = 0;
    for (int i = 0; i < s->n; ++i)
        if (s->type[i] == p->anion_type) idx[m++] = i;
    for (int a = 1; a < m; ++a) {            /* insertion sort on tags */
        const int v = idx[a];
        int b = a - 1;
        while (b >= 0 && s->tag[idx[b]] > s->tag[v]) { idx[b + 1] = idx[b]; --b; }
        idx[b + 1] = v;
    }
    return m;
}

/* sum over the anions of B_ins(r_a, r_c) for the cation at slot ic, in
 * ascending tag order */
static double bias_sum(const or_params *p, const or_state *s, int ic)
{
    int *idx = malloc(sizeof(int) * (size_t)(s->n > 0 ? s->n : 1));
    if (!idx) return NAN;
    const int m = anions_by_tag(p, s, idx);
    double W = 0.0;
    for (int q = 0; q < m; ++q) W += or_bias_B(p, s->x + 3 * idx[q], s->x + 3 * ic);
    free(idx);
    return W;
}

static int pick_rank(const or_state *s, int type, int rank)
{
    /* the atom of the given type whose tag has the given rank (ascending) */
    int best = -1;
    for (int i = 0; i < s->n; ++i) {
        if (s->type[i] != type) continue;
        int below = 0;
        for (int j = 0; j < s->n; ++j)
            if (s->type[j] == type && s->tag[j] < s->tag[i]) ++below;
        if (below == rank) { best = i; break; }
    }
    return best;
}

static void remove_atom(or_state *s, int i)
{
    for (int k = i; k < s->n - 1; ++k) {
        for (int d = 0; d < 3; ++d) {
            s->x[3 * k + d] = s->x[3 * (k + 1) + d];
            s->v[3 * k + d] = s->v[3 * (k + 1) + d];
        }
        s->type[k] = s->type[k + 1];
        s->mol[k] = s->mol[k + 1];
        s->tag[k] = s->tag[k + 1];
        s->flying[k] = s->flying[k + 1];
    }
    s->n--;
}

/* Start of a trial: move choice and proposal (Eqs. 3-4), momenta, the
 * starting Hamiltonian and, for an insertion, the switch-on energy.  On
 * return the flyers are marked (an insertion has appended its ghost pair).
 * Returns 0 if the trial ends here (deletion from an empty box), 1 if the
 * trajectory follows, negative on error. */
/* ------------------------------------------------------------------ */
/* Features of a candidate pair site for the learned proposal.         */
/* ------------------------------------------------------------------ */
#define FEAT_CLIP 1.0e6

static double clipd(double v)
{
    return v > FEAT_CLIP ? FEAT_CLIP : (v < -FEAT_CLIP ? -FEAT_CLIP : v);
}

/* The 31 descriptors of one ion of type T at r, from every non-flying
 * atom (minimum image, all pairs):
 *   [0, 24)  0.1 x Gaussian shell counts of atom types 0..3 in six shells
 *            of width rc/6 up to rc = max cutoff (centres (m + 1/2) rc/6,
 *            standard deviation rc/12), each term tapered by (1 - r^2/rc^2)^2
 *            so that every feature is continuous in the positions;
 *   24       asinh(beta U_C) of the ion at w = 0;
 *   25       asinh(beta |F_C|), the Coulomb force on it at w = 0;
 *   26, 27   asinh(beta U_LJ) at w = 0 and at w = w_max;
 *   28       asinh(beta exp(-kappa_sr w_max) U_C) at w = w_max (Eq. 11);
 *   29, 30   distance to the nearest atom and to the nearest counter-ion,
 *            over rc, capped at 1.
 * Every pair term is scaled by beta and clipped to +-1e6 before it is
 * summed. */
static void ion_features(const or_params *p, const or_state *s, int T, int counter, const double r[3],
                         double out[31])
{
    const double beta = 1.0 / p->kT;
    const double rc = p->rc_lj > p->rc_coul ? p->rc_lj : p->rc_coul;
    const double delta = rc / 6.0, sd = delta / 2.0;
    const double gmax = exp(-p->kappa_sr * p->w_max);
    double shell[24] = {0};
    double uc0 = 0.0, ulj0 = 0.0, uljw = 0.0, ucw = 0.0, F[3] = {0.0, 0.0, 0.0};
    double dmin = INFINITY, dct = INFINITY;
    for (int j = 0; j < s->n; ++j) {
        if (s->flying[j]) continue;
        double d[3], r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            d[c] = minimg(r[c] - s->x[3 * j + c], p->box[c]);
            r2 += d[c] * d[c];
        }
        const double rr = sqrt(r2);
        const int tj = s->type[j];
        if (rr < dmin) dmin = rr;
        if (tj == counter && rr < dct) dct = rr;
        if (rr < rc && tj < 4) {
            const double x = 1.0 - r2 / (rc * rc), taper = x * x;
            for (int m = 0; m < 6; ++m) {
                const double z = (rr - (m + 0.5) * delta) / sd;
                shell[6 * tj + m] += exp(-0.5 * z * z) * taper;
            }
        }
        double ulj, uc, dlj, dc;
        or_pair(p, T, tj, r2, 1.0, &ulj, &uc, &dlj, &dc);
        ulj0 += clipd(beta * ulj);
        uc0 += clipd(beta * uc);
        const double fr = clipd(-beta * dc);          /* radial Coulomb force */
        for (int c = 0; c < 3; ++c) F[c] += fr * d[c] / rr;
        or_pair(p, T, tj, r2 + p->w_max * p->w_max, gmax, &ulj, &uc, &dlj, &dc);
        uljw += clipd(beta * ulj);
        ucw += clipd(beta * uc);
    }
    for (int q = 0; q < 24; ++q) out[q] = 0.1 * shell[q];
    out[24] = asinh(uc0);
    out[25] = asinh(sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]));
    out[26] = asinh(ulj0);
    out[27] = asinh(uljw);
    out[28] = asinh(ucw);
    out[29] = (dmin < rc ? dmin : rc) / rc;
    out[30] = (dct < rc ? dct : rc) / rc;
}

/* Features (64) of the candidate pair site: cation at site[0..2], anion
 * at site[3..5], on the physical state without the flying atoms: 31 for
 * the cation, 31 for the anion, then the pair's separation over rc (capped
 * at 1) and asinh(beta u) of the pair's own energy (3D, unscreened). */
int or_site_features(const or_params *p, const or_state *s, const double site[6], double out[64])
{
    const double beta = 1.0 / p->kT;
    const double rc = p->rc_lj > p->rc_coul ? p->rc_lj : p->rc_coul;
    ion_features(p, s, p->cation_type, p->anion_type, site, out);
    ion_features(p, s, p->anion_type, p->cation_type, site + 3, out + 31);
    double r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double d = minimg(site[c] - site[3 + c], p->box[c]);
        r2 += d * d;
    }
    const double rr = sqrt(r2);
    double ulj, uc, dlj, dc;
    or_pair(p, p->cation_type, p->anion_type, r2, 1.0, &ulj, &uc, &dlj, &dc);
    out[62] = (rr < rc ? rr : rc) / rc;
    out[63] = asinh(clipd(beta * (ulj + uc)));
    return 0;
}

/* Candidate j of trial t: cation and anion uniform in the box, from the
 * counters (t, 4, j, 0) and (t, 4, j, 1). */
static void candidate_site(const or_params *p, uint64_t trial, int j, double site[6])
{
    double a[4], b[4];
    draw4(p, trial, PURPOSE_CAND, (uint64_t)j, a);
    uint64_t c[4] = {trial, PURPOSE_CAND, (uint64_t)j, 1}, k[2] = {p->seed, p->stream}, o[4];
    or_philox4x64(c, k, o);
    for (int q = 0; q < 3; ++q) b[q] = or_u01(o[q]);
    for (int d = 0; d < 3; ++d) {
        site[d] = wrap1(p->box[d] * a[d], p->box[d]);
        site[3 + d] = wrap1(p->box[d] * b[d], p->box[d]);
    }
}

/* log weights of n sites: the proposal's network, or 0 without one */
static int score_sites(const or_params *p, const or_state *s, const or_proposal *prop, int n,
                       const double *sites, double *feat, double *logw)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (int j = 0; j < n; ++j) or_site_features(p, s, sites + 6 * j, feat + 64 * j);
    if (!prop->fn) {
        for (int j = 0; j < n; ++j) logw[j] = 0.0;
        return 0;
    }
    const int rc = prop->fn(prop->ctx, n, feat, logw);
    for (int j = 0; j < n; ++j) logw[j] = prop->scale * fmin(logw[j], prop->cap);
    return rc;
}

int or_trial_begin(const or_params *p, or_state *s, uint64_t trial, int force_move,
                   or_trial_rec *rec, int *ic_out, int *ia_out, int *nf_out)
{
    return trial_begin(p, s, trial, force_move, NULL, rec, ic_out, ia_out, nf_out, NULL);
}

static int trial_begin(const or_params *p, or_state *s, uint64_t trial, int force_move,
                       const or_proposal *prop, or_trial_rec *rec, int *ic_out, int *ia_out, int *nf_out,
                       double *feat_out)
{
    memset(rec, 0, sizeof(*rec));
    rec->trial = (int64_t)trial;
    double u[8];
    draw4(p, trial, PURPOSE_SELECT, 0, u);
    draw4(p, trial, PURPOSE_SELECT, 1, u + 4);
    int nf = p->n_steps;
    if (p->n_steps_max > 0) {
        double un[4];
        draw4(p, trial, PURPOSE_NSTEPS, 0, un);
        nf = p->n_steps_min + (int)floor(un[0] * (double)(p->n_steps_max - p->n_steps_min + 1));
    }
    const int move = force_move ? force_move : (u[0] < 0.5 ? +1 : -1);
    const int Ns = s->nsalt;
    rec->move = move;
    rec->n_salt_before = Ns;
    rec->n_salt_after = Ns;
    rec->n_steps = nf;
    rec->ln_u = log(u[7]);
    *nf_out = nf;
    *ic_out = *ia_out = -1;
    if (move < 0 && Ns == 0) {
        rec->flags |= OR_FLAG_EMPTY;
        rec->ln_ratio = -INFINITY;
        return 0;
    }
    int ic, ia;
    if (move > 0) {
        /* Eq. (4): both flying ions placed uniformly in the box (1/V each);
         * with a learned proposal, one of k uniform candidates chosen with
         * probability proportional to its weight (multiple-try form). */
        if (s->n + 2 > s->cap) return -3;
        double site[6];
        for (int d = 0; d < 3; ++d) { site[d] = p->box[d] * u[1 + d]; site[3 + d] = p->box[d] * u[4 + d]; }
        if (p->bias_alpha > 0.0 && !(prop && prop->k >= 1)) {
            /* Sec. II B 4: the anion at the cation plus an offset drawn from
             * Eq. (14) along each edge */
            for (int d = 0; d < 3; ++d) {
                const double x = or_bias_offset(p, trial, d);
                if (!isfinite(x)) return -9;
                site[3 + d] = site[d] + x;
            }
        }
        if (prop && prop->k >= 1) {
            const int k = prop->k;
            double *sites = malloc(sizeof(double) * 6 * (size_t)k);
            double *feat = malloc(sizeof(double) * 64 * (size_t)k);
            double *logw = malloc(sizeof(double) * (size_t)k);
            if (!sites || !feat || !logw) { free(sites); free(feat); free(logw); return -1; }
            for (int j = 0; j < k; ++j) candidate_site(p, trial, j, sites + 6 * j);
            if (score_sites(p, s, prop, k, sites, feat, logw)) { free(sites); free(feat); free(logw); return -8; }
            /* categorical choice: the first candidate whose running weight
             * exceeds u W (weights relative to the largest) */
            double mx = logw[0], W = 0.0, run = 0.0, us[4];
            for (int j = 1; j < k; ++j) if (logw[j] > mx) mx = logw[j];
            for (int j = 0; j < k; ++j) W += exp(logw[j] - mx);
            draw4(p, trial, PURPOSE_PICK, 0, us);
            const double target = us[0] * W;
            int sel = k - 1;
            for (int j = 0; j < k; ++j) {
                run += exp(logw[j] - mx);
                if (run > target) { sel = j; break; }
            }
            or_mtm_log_factor(+1, k, logw, sel, &rec->ln_proposal);
            for (int q = 0; q < 6; ++q) site[q] = sites[6 * sel + q];
            if (feat_out) memcpy(feat_out, feat + 64 * sel, 64 * sizeof(double));
            free(sites); free(feat); free(logw);
        }
        ic = s->n; ia = s->n + 1;
        for (int d = 0; d < 3; ++d) {
            s->x[3 * ic + d] = wrap1(site[d], p->box[d]);
            s->x[3 * ia + d] = wrap1(site[3 + d], p->box[d]);
        }
        s->type[ic] = p->cation_type; s->type[ia] = p->anion_type;
        s->mol[ic] = -1; s->mol[ia] = -1;
        s->tag[ic] = s->next_tag; s->tag[ia] = s->next_tag + 1;
        s->flying[ic] = 1; s->flying[ia] = 1;
        s->n += 2;
    } else {
        /* Eq. (3): one of the N+1 cations and one of the N+1 anions. */
        ic = pick_rank(s, p->cation_type, (int)floor(u[1] * Ns));
        if (ic < 0) return -4;
        if (p->bias_alpha > 0.0 && !(prop && prop->k >= 1)) {
            /* Eq. (13): the anion with probability B_ins(r_a, r_c) / sum_n
             * B_ins(r_a,n, r_c), the first in ascending tag order whose
             * running sum exceeds u W */
            int *idx = malloc(sizeof(int) * (size_t)s->n);
            if (!idx) return -1;
            const int m = anions_by_tag(p, s, idx);
            double W = 0.0;
            for (int q = 0; q < m; ++q) W += or_bias_B(p, s->x + 3 * idx[q], s->x + 3 * ic);
            const double target = u[2] * W;
            double run = 0.0;
            ia = m > 0 ? idx[m - 1] : -1;
            for (int q = 0; q < m; ++q) {
                run += or_bias_B(p, s->x + 3 * idx[q], s->x + 3 * ic);
                if (run > target) { ia = idx[q]; break; }
            }
            free(idx);
            /* Eq. (16): B_ins / B_del = W / (N + 1) */
            rec->ln_proposal = log(W) - log((double)Ns);
        } else {
            ia = pick_rank(s, p->anion_type, (int)floor(u[2] * Ns));
        }
        if (ia < 0) return -4;
        s->flying[ic] = 1; s->flying[ia] = 1;
    }
    rec->tag_c = s->tag[ic];
    rec->tag_a = s->tag[ia];
    *ic_out = ic; *ia_out = ia;
    if (p->v_ex_edge > 0.0) {
        /* early rejection (supplement): a pair whose anion lies in the cube
         * V_ex centred on the cation is exchanged instantly, a conventional
         * MC move with no trajectory, for insertions and deletions alike (the
         * move type is a function of the pair, so each move and its reverse
         * take the same type) */
        int inside = 1;
        for (int d = 0; d < 3; ++d)
            inside &= fabs(minimg(s->x[3 * ia + d] - s->x[3 * ic + d], p->box[d])) < 0.5 * p->v_ex_edge;
        if (inside) {
            nf = 0;
            *nf_out = 0;
            rec->n_steps = 0;
            rec->flags |= OR_FLAG_INSTANT;
        }
    }

    if (p->momenta) {
        /* carried momenta: the state's own, reversed with probability 1/2
         * at the start of the trajectory; the flyers' drawn afresh */
        double s0, s1;
        reversal_signs(p, trial, &s0, &s1);
        for (int i = 0; i < s->n; ++i) {
            if (s->flying[i]) mb_velocity(p, s, i, trial, PURPOSE_MB, s->v + 3 * i);
            else for (int d = 0; d < 3; ++d) s->v[3 * i + d] *= s0;
        }
    } else if (or_mb_velocities(p, s, trial)) return -5;
    or_energy e;
    /* H at the start: the N-state (ghosts left out) for an insertion, the
     * physical (N+1)-state for a deletion. */
    if (or_compute(p, s, 0.0, move > 0 ? OR_MODE_EXCL : OR_MODE_NEMD, NULL, &e)) return -7;
    /* until the trial completes, dU and dK hold U and K of the start state */
    rec->dU = e.U;
    rec->dK = or_kinetic(p, s);
    rec->H0 = rec->dU + rec->dK;
    if (move > 0) rec->E_switch = u_fly(p, s, p->w_max);
    return 1;
}

int or_trial(const or_params *p, or_state *s, uint64_t trial, int force_move,
             or_trial_rec *rec)
{
    return or_trial_learned(p, s, trial, force_move, NULL, rec, NULL);
}

int or_trial_learned(const or_params *p, or_state *s, uint64_t trial, int force_move,
                     const or_proposal *prop, or_trial_rec *rec, double *feat_out)
{
    const double beta = 1.0 / p->kT;
    const double V = p->box[0] * p->box[1] * p->box[2];
    const int Ns = s->nsalt;
    const int n_orig = s->n;
    int ic, ia, nf;
    if (prop && prop->k < 1) prop = NULL;
    /* the carried momenta before the trial (a rejection restores them) */
    double *v0 = p->momenta ? malloc(3 * (size_t)(n_orig > 0 ? n_orig : 1) * sizeof(double)) : NULL;
    if (p->momenta && !v0) return -1;
    if (v0) memcpy(v0, s->v, 3 * (size_t)n_orig * sizeof(double));
    const int st = trial_begin(p, s, trial, force_move, prop, rec, &ic, &ia, &nf, feat_out);
    if (st <= 0) { free(v0); return st; }
    const int move = rec->move;
    const int n_small = (move > 0) ? Ns : Ns - 1;
    const double H0 = rec->H0;
    double E_switch = rec->E_switch;
    or_energy e;

    double *x0 = malloc(3 * (size_t)s->n * sizeof(double));
    if (!x0) { free(v0); return -1; }
    memcpy(x0, s->x, 3 * (size_t)s->n * sizeof(double));
    double W = 0.0;
    int rc = or_nemd(p, s, move, nf, &W);
    if (rc == -2) {
        /* the rigid-water constraints could not be met (a violent overlap):
         * the trial has no finite outcome and is rejected */
        memcpy(s->x, x0, 3 * (size_t)n_orig * sizeof(double));
        if (move > 0) s->n = n_orig;
        else { s->flying[ic] = 0; s->flying[ia] = 0; }
        rec->dH = NAN;
        rec->flags |= OR_FLAG_NONFINITE;
        rec->ln_ratio = NAN;
        free(x0); free(v0);
        return 0;
    }
    if (rc) { free(x0); free(v0); return -6; }

    if (move > 0) or_compute(p, s, 0.0, OR_MODE_NEMD, NULL, &e);
    else or_compute(p, s, 0.0, OR_MODE_EXCL, NULL, &e);
    const double U1 = e.U, K1 = or_kinetic(p, s);
    if (move < 0) E_switch = -u_fly(p, s, p->w_max);
    if (move < 0 && prop) {
        /* reverse multiple-try weights on the post-trajectory N-state:
         * the removed pair's site first, then k - 1 fresh candidates */
        const int k = prop->k;
        double *sites = malloc(sizeof(double) * 6 * (size_t)k);
        double *feat = malloc(sizeof(double) * 64 * (size_t)k);
        double *logw = malloc(sizeof(double) * (size_t)k);
        if (!sites || !feat || !logw) { free(sites); free(feat); free(logw); free(x0); free(v0); return -1; }
        for (int d = 0; d < 3; ++d) { sites[d] = s->x[3 * ic + d]; sites[3 + d] = s->x[3 * ia + d]; }
        for (int j = 0; j + 1 < k; ++j) candidate_site(p, trial, j, sites + 6 * (j + 1));
        if (score_sites(p, s, prop, k, sites, feat, logw)) {
            free(sites); free(feat); free(logw); free(x0); free(v0);
            return -8;
        }
        or_mtm_log_factor(-1, k, logw, 0, &rec->ln_proposal);
        if (feat_out) memcpy(feat_out, feat, 64 * sizeof(double));
        free(sites); free(feat); free(logw);
    }

    if (move > 0 && p->bias_alpha > 0.0 && !prop) {
        /* Eq. (15): B_del / B_ins = (N + 1) / sum_n B_ins(r_a,n, r_c) over
         * the anions of the (N+1)-state the trajectory reached */
        rec->ln_proposal = log((double)(Ns + 1)) - log(bias_sum(p, s, ic));
    }
    const double dH = (U1 + K1) - H0;
    /* Eqs. (6) and (8) with Lambda_s: ln of (V / (Lambda^3 (N+1)))^2. */
    const double lam3 = p->lambda_s * p->lambda_s * p->lambda_s;
    const double I = 2.0 * log(V / (lam3 * (double)(n_small + 1)));
    double lnR;
    if (move > 0) lnR = -beta * dH + p->beta_mu + I;
    else lnR = -beta * dH - p->beta_mu - I;
    lnR += rec->ln_proposal;
    rec->dU = U1 - rec->dU;
    rec->dK = K1 - rec->dK;
    rec->dH = dH;
    rec->W_prot = W; rec->E_switch = E_switch;
    rec->H1 = U1 + K1;
    rec->dM = (move > 0) ? dH - I / beta : -dH - I / beta;
    rec->ln_ratio = lnR;
    int acc = 0;
    if (!isfinite(dH)) { rec->flags |= OR_FLAG_NONFINITE; acc = 0; }
    else acc = rec->ln_u < lnR;
    rec->accepted = acc;

    if (acc) {
        if (move > 0) {
            s->flying[ic] = 0; s->flying[ia] = 0;
            s->next_tag += 2;
            s->nsalt = Ns + 1;
        } else {
            const int hi = ic > ia ? ic : ia, lo = ic > ia ? ia : ic;
            remove_atom(s, hi);
            remove_atom(s, lo);
            s->nsalt = Ns - 1;
        }
    } else {
        memcpy(s->x, x0, 3 * (size_t)s->n * sizeof(double));
        if (move > 0) s->n = n_orig;
        else { s->flying[ic] = 0; s->flying[ia] = 0; }
    }
    if (p->momenta) {
        /* the end reversal: the state reached keeps its momenta (the new
         * pair's are its fresh draws), or the rejected state its own, each
         * reversed with probability 1/2 */
        double s0, s1;
        reversal_signs(p, trial, &s0, &s1);
        if (acc) for (int q = 0; q < 3 * s->n; ++q) s->v[q] *= s1;
        else for (int q = 0; q < 3 * n_orig; ++q) s->v[q] = s0 * s1 * v0[q];
    }
    rec->n_salt_after = s->nsalt;
    free(x0); free(v0);
    return 0;
}

int or_md_phase(const or_params *p, or_state *s, uint64_t phase, int n_steps, or_trial_rec *rec)
{
    /* Equilibrium sampling between trials, as generalized hybrid Monte
     * Carlo: the momenta are partly refreshed, v <- c v + sqrt(1 - c^2) xi
     * with xi Maxwell-Boltzmann (c = 0: plain hybrid MC), the whole state
     * runs n_steps velocity-Verlet steps in 3D, and the end state is taken
     * with probability min(1, exp(-beta dH)); a rejection keeps the
     * positions and reverses the refreshed momenta.  Each part leaves the
     * canonical distribution of (x, p) invariant.  Rigid waters: the
     * refreshed momenta are restricted to the constraint surface (the
     * velocity constraint, a linear projection that keeps the constrained
     * Maxwell-Boltzmann distribution), and every step constrains positions
     * and velocities as in a trial's trajectory. */
    if (n_steps < 1) return -11;
    const int n = s->n;
    const double beta = 1.0 / p->kT;
    memset(rec, 0, sizeof(*rec));
    rec->move = 2;
    rec->trial = (int64_t)phase;
    rec->n_steps = n_steps;
    rec->n_salt_before = rec->n_salt_after = s->nsalt;
    rec->tag_c = rec->tag_a = -1;
    const double c = p->md_refresh, sc = sqrt(1.0 - c * c);
    for (int i = 0; i < n; ++i) {
        double xi[3];
        mb_velocity(p, s, i, phase, PURPOSE_REFRESH, xi);
        for (int d = 0; d < 3; ++d) s->v[3 * i + d] = c * s->v[3 * i + d] + sc * xi[d];
    }
    if (p->water && or_constrain_velocities(p, s)) return -5;
    double *x0 = malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double *v0 = malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double *F = malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double));
    double *xref = p->water ? malloc(3 * (size_t)(n > 0 ? n : 1) * sizeof(double)) : NULL;
    if (!x0 || !v0 || !F || (p->water && !xref)) { free(x0); free(v0); free(F); free(xref); return -1; }
    memcpy(x0, s->x, 3 * (size_t)n * sizeof(double));
    memcpy(v0, s->v, 3 * (size_t)n * sizeof(double));
    or_energy e;
    if (or_compute(p, s, 0.0, OR_MODE_NEMD, F, &e)) { free(x0); free(v0); free(F); free(xref); return -7; }
    const double U0 = e.U, K0 = or_kinetic(p, s);
    const double h = 0.5 * p->dt;
    int unmet = 0;   /* rigid-water constraints that could not be met */
    for (int k = 0; k < n_steps && !unmet; ++k) {
        for (int i = 0; i < n; ++i) {
            const double m = p->mass[s->type[i]];
            for (int d = 0; d < 3; ++d) s->v[3 * i + d] += h * p->accel * F[3 * i + d] / m;
        }
        if (xref) memcpy(xref, s->x, 3 * (size_t)n * sizeof(double));
        for (int i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d)
                s->x[3 * i + d] = wrap1(s->x[3 * i + d] + p->dt * s->v[3 * i + d], p->box[d]);
        if (xref && or_constrain_positions(p, s, xref)) { unmet = 1; break; }
        if (or_compute(p, s, 0.0, OR_MODE_NEMD, F, &e)) { free(x0); free(v0); free(F); free(xref); return -7; }
        for (int i = 0; i < n; ++i) {
            const double m = p->mass[s->type[i]];
            for (int d = 0; d < 3; ++d) s->v[3 * i + d] += h * p->accel * F[3 * i + d] / m;
        }
        if (p->water && or_constrain_velocities(p, s)) unmet = 1;
    }
    const double U1 = unmet ? NAN : e.U, K1 = or_kinetic(p, s);
    double u[4];
    draw4(p, phase, PURPOSE_MD, 0, u);
    rec->H0 = U0 + K0;
    rec->H1 = U1 + K1;
    rec->dH = rec->H1 - rec->H0;
    rec->dU = U1 - U0;
    rec->dK = K1 - K0;
    rec->ln_ratio = -beta * rec->dH;
    rec->ln_u = log(u[0]);
    int acc = 0;
    if (!isfinite(rec->dH)) rec->flags |= OR_FLAG_NONFINITE;
    else acc = rec->ln_u < rec->ln_ratio;
    rec->accepted = acc;
    if (!acc) {
        memcpy(s->x, x0, 3 * (size_t)n * sizeof(double));
        for (int q = 0; q < 3 * n; ++q) s->v[q] = -v0[q];
    }
    free(x0); free(v0); free(F); free(xref);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Multiple-try factor of the learned proposal.                        */
/* The k candidates of a move carry log weights logw[0..k-1]; for an   */
/* insertion, sel is the chosen one and the factor is                  */
/*     ln(W/k) - logw[sel],     W = sum_j exp(logw[j]);                */
/* for a deletion logw[0] belongs to the removed pair, logw[1..k-1] to  */
/* fresh candidates drawn on the post-trajectory state, and the factor  */
/* is logw[0] - ln(W/k).                                               */
/* ------------------------------------------------------------------ */
int or_mtm_log_factor(int move, int k, const double *logw, int sel, double *out)
{
    if (k < 1 || (move > 0 && (sel < 0 || sel >= k))) return -1;
    double mx = logw[0];
    for (int j = 1; j < k; ++j) if (logw[j] > mx) mx = logw[j];
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += exp(logw[j] - mx);
    const double lnW_over_k = mx + log(acc) - log((double)k);
    *out = (move > 0) ? lnW_over_k - logw[sel] : logw[0] - lnW_over_k;
    return 0;
}
