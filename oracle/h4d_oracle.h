/*
 * h4d_oracle.h -- plain FP64 CPU reference of the hybrid 4D NEMD/MC
 * (H4D) grand-canonical ion-pair exchange of Kim, Belloni & Rotenberg,
 * "Grand-canonical molecular dynamics simulations powered by a hybrid 4D
 * nonequilibrium MD/MC method" (arXiv 2307.11447).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against an
 * independent, slow, obviously correct implementation.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every quantity is FP64.  Single threaded.  Functions return 0 on success
 * and a negative value on a bad argument.
 */
#ifndef H4D_ORACLE_H
#define H4D_ORACLE_H
#include <stdint.h>

#define OR_MAXT 8

/* Physical model and protocol (the parameter names follow the paper). */
typedef struct {
    int32_t n_types;
    int32_t cation_type, anion_type;
    int32_t n_steps;        /* N_f: NEMD steps per trial (Sec. II A)             */
    int32_t n_steps_min;    /* if n_steps_max > 0, N_f ~ U{min..max} per trial   */
    int32_t n_steps_max;
    int32_t water;          /* 1: rigid 3-site waters occupy atoms [0, 3*n_mol)   */
    int32_t use_cells;      /* 1: linked-cell pair search, 0: all pairs           */
    double mass[OR_MAXT], charge[OR_MAXT], sigma[OR_MAXT], eps[OR_MAXT];
    double box[3];
    double kT, dt, w_max, kappa_sr;
    double rc_lj, rc_coul, alpha, ke;
    double beta_mu, lambda_s;
    double d_oh, d_hh;      /* rigid-water geometry                              */
    double accel;           /* acceleration per (force/mass); 1 in reduced units  */
    uint64_t seed, stream;  /* Philox key                                        */
    double bias_xb;         /* bimodal bias of the flyers' separation (Sec.      */
    double bias_alpha;      /* II B 4, Eq. 14): x_b and alpha_b; alpha_b = 0: off */
    int32_t schedule;       /* altitude: 0 Eq. (2); 1 w_max (1 - x^n); 2         */
    double schedule_n;      /* w_max (1 - x)^n (supplement), exponent n           */
    int32_t momenta;        /* 0: fresh Maxwell-Boltzmann momenta every trial; 1: */
                            /* the state's momenta carried into the trajectory    */
                            /* with the symmetric two-end reversal (Sec. II A)    */
    double md_refresh;      /* equilibrium phase: v <- c v + sqrt(1 - c^2) xi     */
    double w_max_ratio;     /* species-specific w_max (supplement): the anion     */
                            /* flies at w_max_ratio times the cation's altitude;  */
                            /* 0 or 1: both at the same altitude                  */
    double v_ex_edge;       /* early rejection (supplement): edge of the cube V_ex */
                            /* around the flying cation; a pair whose anion lies  */
                            /* inside is exchanged instantly (no trajectory);     */
                            /* 0: off                                             */
} or_params;

/* Configuration.  Arrays are owned by the caller and sized to cap. */
typedef struct {
    int32_t n, cap, nsalt, n_mol;
    int64_t next_tag;
    double *x;          /* 3*cap, wrapped into [0, L)                      */
    double *v;          /* 3*cap                                           */
    int32_t *type;      /* cap                                             */
    int32_t *mol;       /* cap, molecule id or -1                          */
    int64_t *tag;       /* cap, unique, never reused                       */
    int32_t *flying;    /* cap, 1 for the two exchanged ions during a trial */
} or_state;

/* One trial's outcome (move: +1 insertion, -1 deletion). */
typedef struct {
    int32_t move, accepted, n_salt_before, n_salt_after, n_steps, flags;
    int64_t trial, tag_c, tag_a;
    double dH, dU, dK, W_prot, E_switch, dM, ln_ratio, ln_u, ln_proposal, H0, H1;
} or_trial_rec;

#define OR_FLAG_EMPTY     1u   /* deletion attempted with no salt pair present */
#define OR_FLAG_NONFINITE 2u   /* dH not finite: rejected                       */
#define OR_FLAG_INSTANT  16u   /* pair inside V_ex: instantaneous exchange      */

/* Energy modes. */
#define OR_MODE_NEMD   0   /* flyers at altitude w, 4D distance, screened Coulomb */
#define OR_MODE_EXCL   1   /* every pair that involves a flyer is left out         */
#define OR_MODE_FLY    2   /* only pairs that involve at least one flyer           */

typedef struct {
    double U, U_lj, U_c, virial, dUdw;
} or_energy;

/* Counter-based generator Philox4x64-10 (Salmon et al., SC'11). */
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_u01(uint64_t bits);

/* Pair energy and radial derivative at 4D distance s (squared: s2). */
int or_pair(const or_params *p, int ti, int tj, double s2, double g,
            double *u_lj, double *u_c, double *dlj_ds, double *dc_ds);

/* Energy (and optionally forces F[3n]) at altitude w in the given mode. */
int or_compute(const or_params *p, const or_state *s, double w, int mode,
               double *F, or_energy *e);

/* Maxwell-Boltzmann velocities for trial t, keyed by atom tag. */
int or_mb_velocities(const or_params *p, or_state *s, uint64_t trial);

/* Rigid-water constraints: positions (iterated to convergence) after a
 * drift from reference xref, with the matching velocity correction; and the
 * velocity projection onto the constraint tangent space. */
int or_constrain_positions(const or_params *p, or_state *s, const double *xref);
int or_constrain_velocities(const or_params *p, or_state *s);

/* Kinetic energy of non-flying atoms. */
double or_kinetic(const or_params *p, const or_state *s);

/* Altitude schedule w_k (Eq. 2) for move (+1 ins / -1 del), k = 0..nf. */
double or_altitude(const or_params *p, int move, int k, int nf);

/* The NEMD trajectory of one trial with the flyers already marked:
 * velocity Verlet from the current x, v for nf steps.  Returns the
 * protocol work W (sum of altitude increments of U_fly). */
int or_nemd(const or_params *p, or_state *s, int move, int nf, double *W);

/* Start of a trial: proposal, momenta, H_start (rec->H0) and, for an
 * insertion, the switch-on energy (rec->E_switch).  Returns 1 if the
 * trajectory follows, 0 if the trial ends (empty deletion), <0 on error. */
int or_trial_begin(const or_params *p, or_state *s, uint64_t trial, int force_move,
                   or_trial_rec *rec, int *ic, int *ia, int *nf);

/* One full trial (move choice, proposal, momenta, NEMD, Metropolis,
 * commit or rollback).  force_move: 0 = random, +1 / -1 forced. */
int or_trial(const or_params *p, or_state *s, uint64_t trial, int force_move,
             or_trial_rec *rec);

/*
 * Learned proposal (multiple-try form of the uniform pair insertion of
 * Eq. 4; a bias on the initial flying-ion positions corrected in the
 * Rosenbluth form of Sec. II B 4, Eqs. 15-16).  Log weights are
 * lw = scale min(logit, cap).  An insertion draws k uniform candidate pair
 * sites (counters (t, 4, j, 0/1)), weighs them by exp(lw) on the state
 * before the trajectory and picks one with probability proportional to its
 * weight (uniform (t, 5, 0, 0)); the ratio gains ln(W/k) - lw(chosen).  A
 * deletion weighs the removed pair's site and k - 1 fresh candidates on the
 * state after the trajectory (pair removed); the ratio gains
 * lw(removed) - ln(W/k).  Exact for any weights; k = 1, scale 0 or equal
 * weights give the uniform proposal.
 */
typedef int (*or_logit_fn)(void *ctx, int n, const double *features /* n x 64 */, double *logits /* n */);
typedef struct {
    int32_t k;          /* candidates per move (>= 1)                     */
    or_logit_fn fn;     /* network; NULL: every logit 0                   */
    void *ctx;
    double cap;         /* log weight = scale * min(logit, cap)           */
    double scale;
} or_proposal;

/* The 64 features of a candidate pair site (cation site[0..2], anion
 * site[3..5]) on the physical state without the flying atoms. */
int or_site_features(const or_params *p, const or_state *s, const double site[6], double out[64]);

/* Bimodal bias (Sec. II B 4): b_ins of Eq. (14) for the anion's offset x
 * (minimum image, |x| <= L/2) along an edge of length L, and B_ins of
 * Eq. (12) for an anion at xa and a cation at xc. */
double or_bias_b(double x, double L, double xb, double alpha);
double or_bias_B(const or_params *p, const double xa[3], const double xc[3]);
/* The anion offset of an insertion along edge d (a draw from Eq. 14). */
double or_bias_offset(const or_params *p, uint64_t trial, int d);

/* A trial with the learned proposal (prop NULL: uniform).  feat_out (may
 * be NULL) receives the features of the inserted or removed pair's site. */
int or_trial_learned(const or_params *p, or_state *s, uint64_t trial, int force_move,
                     const or_proposal *prop, or_trial_rec *rec, double *feat_out);

/* ln of the multiple-try factor for log weights logw[0..k-1] (insertion:
 * sel is the chosen candidate; deletion: logw[0] is the removed pair). */
/* Momenta of a new state: every atom's velocity drawn from the
 * Maxwell-Boltzmann distribution (counter 0 of its own stream). */
int or_init_velocities(const or_params *p, or_state *s);

/* Equilibrium phase between trials (generalized hybrid MC): partial
 * momentum refresh, n_steps velocity-Verlet steps of the whole state in 3D,
 * Metropolis test on exp(-beta dH); a rejected phase restores the positions
 * and reverses the refreshed momenta.  rec->move = 2, rec->trial = phase. */
int or_md_phase(const or_params *p, or_state *s, uint64_t phase, int n_steps, or_trial_rec *rec);

int or_mtm_log_factor(int move, int k, const double *logw, int sel, double *out);

#endif
