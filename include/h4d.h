/*
 * h4d.h -- C ABI of the MI355X (gfx950) library for hybrid 4D
 * nonequilibrium MD/MC (H4D) grand-canonical ion-pair exchange, after
 * Kim, Belloni & Rotenberg, "Grand-canonical molecular dynamics simulations
 * powered by a hybrid 4D nonequilibrium MD/MC method" (arXiv 2307.11447).
 *
 * One call of h4d_run_nemd_trial is one exchange attempt of the paper's
 * GCMD cycle (Sec. II A, Fig. 1): choose insertion or deletion of a
 * cation-anion pair, fly the pair along the fourth coordinate w with the
 * constant-velocity schedule of Eq. (2) during an NVE velocity-Verlet
 * trajectory, and accept or reject with the Metropolis ratio of
 * Eqs. (6) and (8).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an h4d_status; none aborts or throws.  On an
 *    error, h4d_last_error() returns a message (thread local, valid until
 *    the next call on the same thread).
 *  - Host arrays passed in are read during the call and copied; the
 *    library never keeps a pointer to caller memory.  Device memory is
 *    allocated and owned by the library and released by the matching
 *    destroy call.
 *  - All GPU work of a handle is enqueued on the hipStream_t given at
 *    creation (NULL: the default stream).  A call that returns host results
 *    synchronises that stream only.
 *  - One host thread may use a handle at a time.
 *  - Units are the caller's: coulomb_k is the Coulomb constant
 *    (k_e q_i q_j / r), accel converts force/mass into acceleration
 *    (1 in reduced units; 4.184e-4 A/fs^2 per (kcal/mol/A)/amu in real
 *    units), kT the thermal energy.
 *  - Results depend only on the starting state, the parameters, the seed
 *    and the trial index: all random numbers come from the counter-based
 *    generator Philox4x64-10 keyed by (seed, stream) with counters
 *    (trial, purpose, tag, 0); the order of atoms in memory is not
 *    observable.
 */
#ifndef H4D_H
#define H4D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define H4D_MAX_TYPES 8

/* Status codes. */
#define H4D_OK          0
#define H4D_EINVAL     -1   /* bad argument (message says which)              */
#define H4D_ENOMEM     -2   /* device allocation failed                        */
#define H4D_EHIP       -3   /* a HIP runtime call failed                       */
#define H4D_ECAPACITY  -4   /* atom capacity exhausted                         */
#define H4D_ENONFINITE -5   /* reserved: non-finite trials are rejected instead */
#define H4D_ENODEV     -6   /* no usable gfx950 device                         */

/* Trial moves. */
#define H4D_MOVE_AUTO    0  /* insertion or deletion with probability 1/2    */
#define H4D_MOVE_INSERT  1
#define H4D_MOVE_DELETE -1
#define H4D_MOVE_MD      2  /* record of an equilibrium phase (h4d_run_md)  */

/* Arithmetic of the pair pass. */
#define H4D_PREC_FP64 0     /* everything in FP64                               */
#define H4D_PREC_FP32 1     /* FP32 pair arithmetic on 32-bit fixed-point
                               coordinates; FP64 positions, velocities,
                               energies, work and Metropolis ratio             */

/* Trial flags. */
#define H4D_FLAG_EMPTY     0x1u  /* deletion drawn with no pair present: rejected */
#define H4D_FLAG_NONFINITE 0x2u  /* dH not finite (a violent overlap blew up the
                                    trajectory): rejected, state rolled back      */
#define H4D_FLAG_RETRIED   0x4u  /* the trial was recomputed after a list resize   */
#define H4D_FLAG_IDLE      0x8u  /* internal: a box of a batch with no trial left */
#define H4D_FLAG_INSTANT   0x10u /* the pair lay in V_ex: exchanged instantly     */

/*
 * Model and protocol.  Types index the per-type tables; pair parameters
 * follow Lorentz-Berthelot mixing (Sec. II D 2).
 *   Lennard-Jones, Eq. (19): truncated and shifted at rc_lj, force not
 *     shifted.
 *   Coulomb: damped shifted force (erfc-screened, real space only; the
 *     Wolf-family option of Sec. II B 2) with damping dsf_alpha and cutoff
 *     rc_coul; between a flying and a non-flying atom it is multiplied by
 *     exp(-kappa_sr w) (Eq. 11).
 *   A pair that involves exactly one flying atom uses the 4D distance
 *     sqrt(r^2 + w^2) (Sec. I, Sec. II C); both cutoffs apply to it.
 *   w follows Eq. (2): w_max -> 0 for an insertion, 0 -> w_max for a
 *     deletion, in n_steps steps of dt (or one of the supplement's
 *     variable-velocity schedules, field schedule); the flying ions stay
 *     fixed in 3D (trick (i) of Sec. II B).
 *   water = 1: the first 3*n_mol atoms are rigid 3-site waters (O, H, H),
 *     bond lengths d_oh and d_hh, intramolecular pairs excluded.
 */
typedef struct h4d_params {
    int32_t n_types;
    int32_t cation_type, anion_type;
    int32_t n_steps;            /* N_f                                         */
    int32_t n_steps_min;        /* n_steps_max > 0: N_f ~ U{min..max} per trial */
    int32_t n_steps_max;
    int32_t water;
    int32_t precision;          /* H4D_PREC_*                                   */
    int32_t capacity;           /* maximum atoms per box (0: the box's
                                   n_atoms + max(1024, n_atoms / 8))           */
    int32_t rebuild_every;      /* neighbour-list rebuild interval (0: auto)   */
    int32_t lanes_per_atom;     /* lanes per atom in list traversals: 4, 8, 16
                                   (0: chosen from the atom count)              */
    int32_t schedule;           /* altitude schedule: 0 constant vertical
                                   velocity (Eq. 2); 1 w_max (1 - x^n); 2
                                   w_max (1 - x)^n, x = k / n_steps for an
                                   insertion, the time reversal for a deletion */
    double mass[H4D_MAX_TYPES], charge[H4D_MAX_TYPES];
    double sigma[H4D_MAX_TYPES], eps[H4D_MAX_TYPES];
    double box[3];              /* orthorhombic edges; each >= 2 max cutoff     */
    double kT, dt, w_max, kappa_sr;
    double rc_lj, rc_coul, dsf_alpha, coulomb_k;
    double beta_mu;             /* beta * mu_salt                               */
    double lambda_s;            /* sqrt(Lambda_+ Lambda_-), Eq. (6)             */
    double skin;                /* Verlet-list skin                              */
    double d_oh, d_hh;          /* rigid-water geometry                          */
    double accel;               /* acceleration per force/mass                   */
    uint64_t seed, stream;      /* Philox key (box b of a batch: seed,
                                   stream + b)                                  */
    double bias_xb, bias_alpha; /* bimodal bias of the flying pair (Sec. II B 4,
                                   Eqs. 12-16), see h4d_set_bias; bias_alpha = 0:
                                   the uniform placement of Eq. (4)             */
    double schedule_n;          /* exponent n >= 1 of schedules 1 and 2         */
    int32_t momenta;            /* 0: every trial draws fresh Maxwell-Boltzmann
                                   momenta; 1: trials carry the state's momenta
                                   with the symmetric two-end reversal (Sec.
                                   II A), to alternate with h4d_run_md (rigid
                                   waters' momenta stay on the constraint
                                   surface).  Speculative replicas start from
                                   the chain's momenta times the reversal
                                   signs of the trials before theirs         */
    double md_refresh;          /* c in [0, 1] of the equilibrium phase's
                                   momentum refresh, see h4d_run_md             */
    double w_max_ratio;         /* species-specific w_max (the supplement's
                                   remedy for overlapping flyers): the anion
                                   flies at r_w = w_max_ratio times the cation's
                                   altitude all along the schedule (w_max is
                                   the cation's), both reaching w = 0 together;
                                   their own pair sits at (w_c - w_a)^2 and
                                   Eq. 11 screening takes the flyers' mean
                                   altitude (Sec. II B 2).  0 or 1: one
                                   altitude for both                           */
    double v_ex_edge;           /* early rejection (the supplement's
                                   instantaneous exchange): edge of the cube
                                   V_ex centred on the flying cation.  A pair
                                   whose anion lies inside, on insertion or
                                   deletion alike, is exchanged with no
                                   trajectory (n_steps = 0, H4D_FLAG_INSTANT):
                                   the Metropolis test of Eqs. 6 and 8 on the
                                   potential-energy change alone.  0: off; not
                                   with the learned proposal                    */
} h4d_params;

/* One trial (move +1 insertion, -1 deletion). */
typedef struct h4d_trial {
    int32_t move, accepted, n_salt_before, n_salt_after, n_steps;
    uint32_t flags;
    int32_t n_atoms;    /* atoms integrated (state size at the start)          */
    int32_t n_rebuilds; /* neighbour-list builds during the trajectory          */
    int64_t trial, tag_c, tag_a;
    double dH;          /* H_end - H_start, H = U_physical + K_non-flying          */
    double dU, dK;
    double W_prot;      /* protocol work: sum of altitude increments of U_fly     */
    double E_switch;    /* U_fly switched on at w_max (insertion) / off (deletion) */
    double dM;          /* insertion-signed work of Eqs. (6)/(8)                   */
    double ln_ratio;    /* ln of the Metropolis ratio                              */
    double ln_u;        /* ln of the uniform it is compared with                   */
    double ln_proposal; /* proposal factor (0 for the uniform proposal)            */
    double H0, H1;
} h4d_trial;

/* Observables of the current state (Eq. 1 statistics over the trials run). */
typedef struct h4d_observables {
    int64_t n_atoms, n_salt, n_trials, n_ins, n_ins_acc, n_del, n_del_acc;
    double U, U_lj, U_coul, virial, pressure_virial;
    double N_mean, N2_mean, chi;   /* running <N_salt>, <N_salt^2>, Var/<N>     */
} h4d_observables;

typedef struct h4d_system h4d_system;   /* opaque, library-owned */

/*
 * Create a system from a host configuration.
 *   pos[3*n_atoms] positions (wrapped into the box), type[n_atoms],
 *   mol[n_atoms] (molecule id, -1 for ions), tag[n_atoms] (unique,
 *   ascending in array order).  n_salt cations and n_salt anions must be
 *   present.  With water = 1 the waters come first, molecule k at atoms
 *   3k, 3k+1, 3k+2 (O, H, H).
 *   hip_stream: a hipStream_t or NULL.
 * The neighbour list is built before return.  *out receives the handle.
 */
int32_t h4d_init_system(const h4d_params *params, int32_t n_atoms, int32_t n_salt,
                        int32_t n_mol, const double *pos, const int32_t *type,
                        const int32_t *mol, const int64_t *tag, void *hip_stream,
                        h4d_system **out);

/*
 * Create a batch of independent boxes (replicas of uneven size and density)
 * that run their trials together.  Every box has its own Markov chain: box b
 * draws its random numbers from Philox key (seed, stream + b), so box b of a
 * batch reproduces, trial for trial, a single system created with
 * box = box_edges[3b..3b+2] and stream + b.  Model parameters are shared;
 * params->box is ignored.
 *   box_edges[3*n_boxes]   orthorhombic edges of each box (each >= 2 max cutoff);
 *   n_atoms[n_boxes], n_salt[n_boxes];
 *   pos, type, tag: the boxes' configurations one after another (box 0's
 *   n_atoms[0] atoms first), same conventions as h4d_init_system.
 * Every box must have >= 3 list cells per edge, or every box fewer.  No
 * rigid water (water = 0).
 */
int32_t h4d_init_batch(const h4d_params *params, int32_t n_boxes, const double *box_edges,
                       const int32_t *n_atoms, const int32_t *n_salt, const double *pos,
                       const int32_t *type, const int64_t *tag, void *hip_stream,
                       h4d_system **out);

/* Number of boxes of a handle (1 for h4d_init_system). */
int32_t h4d_num_boxes(const h4d_system *sys);

/* Rebuild the cell and Verlet lists of the current state (cells of edge
 * >= max cutoff + skin; all pairs when a box edge holds fewer than 3). */
int32_t h4d_build_neighbors(h4d_system *sys);

/*
 * Run exchange trials on the device.  Trial t (the handle's counter, then
 * t+1, ...) draws its move, sites and momenta from the generator, runs the
 * NEMD trajectory and the Metropolis test (Eqs. 6 and 8 with Lambda_s),
 * and commits or rolls back.  out[n] receives the records (host memory).
 * move forces every trial's direction (H4D_MOVE_*).  Lists that overflow
 * during a trial grow and the trial is recomputed (H4D_FLAG_RETRIED), with
 * the same result.  An insertion into a box at its atom capacity returns
 * H4D_ECAPACITY before any device state changes: the state, the running sums
 * and the trial counter stay as they were, so the next call runs the same
 * trial index (a deletion fits).
 */
int32_t h4d_run_nemd_trial(h4d_system *sys, int32_t move, h4d_trial *out);
int32_t h4d_run_trials(h4d_system *sys, int32_t n, int32_t move, h4d_trial *out);

/*
 * Equilibrium phase between trials (Sec. II A, Fig. 1: equilibrium MD samples
 * configurations between exchange trials), one in every box: the state's
 * momenta are partly refreshed, v <- c v + sqrt(1 - c^2) xi with xi
 * Maxwell-Boltzmann and c = md_refresh (c = 0: plain hybrid MC), the whole
 * state runs n_steps velocity-Verlet steps in 3D (no flyers), and the end
 * state is taken with probability min(1, exp(-beta dH)); a rejected phase
 * keeps the positions and reverses the refreshed momenta (generalized
 * hybrid MC, exact for the canonical distribution at any dt).  Phase p of a
 * box draws from the generator with counter p (its own sequence, apart from
 * the trials').  The momenta stay with the state: trials with momenta = 1
 * start from them, and h4d_get_state returns them.  out (host, may be NULL)
 * receives one record per box: move = H4D_MOVE_MD, trial = the phase index,
 * dH, dU, dK, H0, H1, ln_ratio = -beta dH, ln_u, accepted.  On a speculative
 * handle the phase runs on the first replica and the others take its state
 * (every record is that replica's).  Rigid waters: the refreshed momenta are
 * restricted to the constraint surface (the velocity constraint, which keeps
 * the constrained Maxwell-Boltzmann distribution) and every step constrains
 * positions and velocities as a trial's trajectory does; a phase whose
 * constraints cannot be met is rejected (H4D_FLAG_NONFINITE).  n_steps >= 1.
 */
int32_t h4d_run_md(h4d_system *sys, int32_t n_steps, h4d_trial *out);

/*
 * Run trials_per_box more trials in every box of a batch.  All boxes run
 * their current trial in one round of launches (one graph, each box with its
 * own N_f and move); a box that must recompute a trial after a list resize
 * does so in the next round while the others go on.  out (host, may be
 * NULL) receives n_boxes * trials_per_box records, box-major:
 * out[b * trials_per_box + t].  Also accepts a single-box handle.
 */
int32_t h4d_run_batch(h4d_system *sys, int32_t trials_per_box, int32_t move, h4d_trial *out);

/*
 * Speculative trials of ONE chain (the trial sequence of Sec. II A, Fig. 1,
 * unchanged).  A trial's outcome depends only on the state it starts from
 * and on its index (every random number is keyed by the index), and a
 * rejected trial leaves the positions unchanged.  So `replicas` copies of the
 * state can run trials t, t+1, ..., t+replicas-1 side by side: the results up
 * to and including the first accepted trial are the chain's, exactly as if
 * run one after another; the later ones are discarded and every copy takes
 * the state after the chain's last kept trial.  With carried momenta
 * (h4d_params.momenta = 1) a rejected trial reverses the momenta by the
 * product of its two reversal signs: copy b starts from the chain's momenta
 * times the products of trials t .. t+b-1, and a round in a box with no salt
 * (where a drawn deletion makes no move) runs the first copy alone.  With
 * acceptance probability p, a round yields about (1 - (1-p)^replicas) / p
 * trials.
 *
 * h4d_init_speculative: the handle, from one configuration with the same
 * arguments and conventions as h4d_init_system (rigid water included;
 * 1 <= replicas <= 64; every replica uses Philox key (seed, stream)).  It is a batch of `replicas` boxes: the
 * observables, state, timing and autotuning calls work on it (every box
 * holds the chain's state between calls; h4d_run_batch runs the same trial
 * in every replica, which keeps them equal, and leaves the chain's
 * statistics out).
 *
 * h4d_run_speculative: n_trials more trials of the chain; out[n_trials]
 * (host) receives their records (field `trial` runs on from the chain's
 * counter) and *rounds (may be NULL) the number of rounds used.  move forces
 * every trial's direction (H4D_MOVE_*).
 */
int32_t h4d_init_speculative(const h4d_params *params, int32_t replicas, int32_t n_atoms, int32_t n_salt,
                             int32_t n_mol, const double *pos, const int32_t *type, const int32_t *mol,
                             const int64_t *tag, void *hip_stream, h4d_system **out);
int32_t h4d_run_speculative(h4d_system *sys, int32_t n_trials, int32_t move, h4d_trial *out, int32_t *rounds);

/* FP64 energies and virial of the current state, plus the running
 * particle-number statistics of the trials run so far (box 0, or box `box`
 * of a batch). */
int32_t h4d_sample_observables(h4d_system *sys, h4d_observables *out);
int32_t h4d_box_observables(h4d_system *sys, int32_t box, h4d_observables *out);

/* Copy the current state to host arrays of length >= cap (positions 3*cap).
 * Any pointer may be NULL.  *n receives the number of atoms.  vel: the
 * state's own momenta (with momenta = 1, after set-up and after an
 * equilibrium phase); after a trial with fresh momenta, the momenta its
 * trajectory ended with. */
int32_t h4d_get_state(h4d_system *sys, int32_t cap, int32_t *n, int32_t *n_salt,
                      double *pos, double *vel, int32_t *type, int32_t *mol, int64_t *tag);
/* The same for box `box` of a batch. */
int32_t h4d_get_box_state(h4d_system *sys, int32_t box, int32_t cap, int32_t *n,
                          int32_t *n_salt, double *pos, double *vel, int32_t *type,
                          int32_t *mol, int64_t *tag);

/*
 * Checkpoint and resume of one chain (a single-box or a speculative handle;
 * not a batch).  The chain has no hidden
 * generator state: every random number is a Philox draw keyed by (seed,
 * stream) and counted by the trial index, the equilibrium-phase index and the
 * ions' tags (the trial sequence of Sec. II A and the phase of Fig. 1).  So
 * the atoms (h4d_get_state) and the fields below are all a new handle needs
 * to continue where this one stands, with the same records: bitwise at the
 * same launch shape, list capacities and rebuild interval, which the
 * checkpoint carries.
 *
 * Resume: h4d_init_system(&ck.params, n, n_salt, n_mol, pos, type, mol, tag,
 * stream, &sys) with the arrays of h4d_get_state, or h4d_init_speculative
 * with the same arrays, then h4d_restore_checkpoint(sys, &ck, n, vel).  A
 * chain saved from one kind of handle resumes on the other; its records are
 * then those of the uninterrupted run as the speculative trials guarantee
 * (bitwise with a fixed rebuild interval).  A learned proposal is not part
 * of the checkpoint: save its network with h4d_mlp_get_weights and apply it
 * again with h4d_set_proposal.
 */
typedef struct h4d_checkpoint {
    h4d_params params;        /* the parameters in force (setters included)  */
    uint64_t trial;           /* index of the next trial                      */
    uint64_t md_phases;       /* equilibrium phases run (their counter)       */
    int64_t next_tag;         /* tag the next inserted cation takes           */
    int32_t lanes_per_atom;   /* step-kernel launch shape in force: 4, 8, 16  */
    int32_t rebuild_every;    /* list rebuild interval in force               */
    int32_t clean_trials;     /* automatic interval: trials since the last
                                 change                                       */
    int32_t interval_tuned;   /* 1: h4d_autotune fixed the interval           */
    int32_t nbr_cap, cell_cap;/* list capacities reached                      */
    int32_t has_velocities;   /* 1: the state carries its own momenta (the vel
                                 of h4d_get_state), required by the restore   */
    int32_t reserved;
    int64_t n_trials, n_ins, n_ins_acc, n_del, n_del_acc;
    double N_sum, N2_sum;     /* running sums behind h4d_sample_observables   */
} h4d_checkpoint;

/* Fill *ck from a single-box or speculative handle (H4D_EINVAL for a
 * batch: see h4d_save_box_checkpoint).  Synchronizes the handle's stream. */
int32_t h4d_save_checkpoint(h4d_system *sys, h4d_checkpoint *ck);
/* Apply *ck to a handle just created from the checkpoint's parameters and
 * the state saved with it.  n_atoms: the state's atom count (checked); vel:
 * host array n_atoms x 3 of the state's momenta (required when
 * ck->has_velocities, else ignored; copied to every replica).  Errors: H4D_EINVAL for a
 * handle whose seed, stream, precision, momenta mode, type count or water
 * flag differ from the checkpoint's, an atom-count mismatch, next_tag not
 * above every tag of the state, or invalid shape or capacities; the handle
 * is then unchanged.  Rebuilds the lists. */
int32_t h4d_restore_checkpoint(h4d_system *sys, const h4d_checkpoint *ck, int32_t n_atoms,
                               const double *vel);
/* The same for box `box` of a batch, each box a chain of its own (box 0 of a
 * single-box or speculative handle).  The saved record carries the box's own
 * edges (params.box) and Philox stream (params.stream = the batch's stream +
 * box), so it also resumes as a single-box handle; a batch resumes from its
 * boxes' records with h4d_init_batch(&ck[0].params, ...) and one restore per
 * box.  The restore checks the box's edges and stream as well. */
int32_t h4d_save_box_checkpoint(h4d_system *sys, int32_t box, h4d_checkpoint *ck);
int32_t h4d_restore_box_checkpoint(h4d_system *sys, int32_t box, const h4d_checkpoint *ck,
                                   int32_t n_atoms, const double *vel);

/* Chemical potential beta * mu_salt of the following trials (Eqs. 6, 8). */
int32_t h4d_set_beta_mu(h4d_system *sys, double beta_mu);

/* Set the next trial index of every box (default 0). */
int32_t h4d_set_trial_index(h4d_system *sys, uint64_t trial);

/*
 * Bimodal bias of the flying pair's separation (Sec. II B 4, Eqs. 12-16),
 * for the following trials (alpha_b = 0: off).  An insertion places the
 * cation uniformly and the anion at an offset drawn along each edge from
 * Eq. (14): Gaussians of exponent alpha_b at +-x_b, normalised on the edge,
 * the offset taken as the minimum image (Philox counters (trial, 6,
 * 4 attempt + edge, 0): a uniform picks the sign, Box-Muller the normal, a
 * draw beyond half an edge is redrawn).  A deletion picks the cation by
 * rank as before and the anion with probability B_ins(r_a, r_c) / W in tag
 * order (Eq. 13), W the sum over the anions of B_ins = V prod b (Eq. 12).
 * ln R gains ln((N+1) / W) for an insertion (W over the anions of the state
 * its trajectory reached) and ln(W / (N+1)) for a deletion (W over those of
 * its start state), Eqs. (15)-(16); the factor is reported in
 * h4d_trial.ln_proposal.  Requires x_b + 6 / sqrt(2 alpha_b) <= half of
 * every box edge; exclusive with the learned proposal.
 */
int32_t h4d_set_bias(h4d_system *sys, double x_b, double alpha_b);

/*
 * Early rejection (the supplement's instantaneous exchange of a pair in
 * contact) from the next trial on: v_ex_edge is the edge of the cube V_ex
 * centred on the flying cation, as h4d_params.v_ex_edge (0: off).  H4D_EINVAL
 * for a negative or non-finite edge, or with the learned proposal set.
 */
int32_t h4d_set_early_rejection(h4d_system *sys, double v_ex_edge);

/*
 * Test hook (single-box handles): forces and FP64 energy of the current state with atoms
 * flying[0], flying[1] (-1: none) lifted to altitude w, as in the NEMD pass
 * (an anion among them to w_max_ratio * w when that is set).
 * forces[3*n] (host) receives F on every non-flying atom (0 on flyers),
 * computed in the handle's precision; energy[3] receives U, U_lj, U_coul.
 */
int32_t h4d_forces_at(h4d_system *sys, const int32_t flying[2], double w,
                      double *forces, double *energy);

/*
 * Kernel timing for roofline measurements.  While enabled, every launch of
 * the fused NEMD step kernel is bracketed by HIP events on the handle's
 * stream (hipExtLaunchKernelGGL); h4d_get_timing returns the accumulated
 * device time of those launches, their count, the atoms they integrated, and
 * the mean Verlet-list length of the current state.
 */
typedef struct h4d_timing {
    int64_t step_launches;
    int64_t retries;       /* trials recomputed with a shorter rebuild interval */
    double step_ms;        /* summed device time of the step kernel            */
    double mean_nbr;       /* mean list entries per atom, current state        */
    int32_t rebuild_every; /* list rebuild interval (steps)                     */
    int32_t nbr_cap;       /* list capacity per atom                           */
    int32_t lanes;         /* lanes per atom                                   */
    int32_t cell_cap;      /* atoms per cell capacity                          */
    double atom_launches;  /* atoms the timed step launches integrated: over
                              every trajectory timed, (N_f + 1) launches times
                              the atoms of its state                           */
    int64_t nonfinite;     /* trials rejected as non-finite (a trajectory that
                              blew up) since the handle was created, every box
                              and the autotuner's trials included              */
    int64_t retries_total; /* trials recomputed since the handle was created   */
    int32_t nt_lists;      /* 1: the FP32 pair pass loads its list indices
                              non-temporally, as it does when a step's list
                              entries and atom state (estimated from the
                              densities at set-up) exceed the 256 MB Infinity
                              Cache (the results are the same either way)     */
    int32_t reserved;
} h4d_timing;

int32_t h4d_set_timing(h4d_system *sys, int32_t on);
int32_t h4d_get_timing(h4d_system *sys, h4d_timing *out);

/*
 * How the FP32 pair pass (Sec. II A: the force on every atom at each step of
 * the trajectory) loads its list indices: mode -1 by the rule of
 * h4d_timing.nt_lists (non-temporal when a step's list entries and atom
 * state exceed the 256 MB Infinity Cache; the default), 0 cached, 1
 * non-temporal.  Records and states are bitwise the same in every mode; only
 * the time differs.  H4D_EINVAL for a null handle or another mode.
 */
int32_t h4d_set_list_loads(h4d_system *sys, int32_t mode);

/*
 * Autotuner of the launch shape: runs `trials` trials (per box) with each
 * lanes-per-atom choice (4, 8, 16) of the list traversals and keeps the one
 * with the least wall time per atom-step; then the number of blocks that
 * share a cell in the list build (1 to 16); then, unless the parameters fix
 * the rebuild interval, times base intervals of 1/4 to 2 times the
 * automatic one and keeps the best for the handle's life (a trial whose
 * fast-atom list overflows is still recomputed with a shorter one).
 * Returns the choices in *lanes_out and *rebuild_out and the best time in
 * *ns_per_atom_step (each may be NULL).  The trials are ordinary trials of
 * the handle's chains (they advance the trial counters and the
 * statistics).  Trajectories depend on the interval only through the
 * summation order, so a tuned handle is reproducible given its choices.
 */
int32_t h4d_autotune(h4d_system *sys, int32_t trials, int32_t *lanes_out, int32_t *rebuild_out,
                     double *ns_per_atom_step);

/*
 * MEASUREMENT ONLY, not part of the method: the stream-copy probe that
 * calibrates the benchmark's hardware byte counters (no handle needed).  It
 * copies `bytes` bytes between two device buffers with a plain
 * 16-byte-per-lane copy kernel `reps` times and returns the mean kernel time
 * in *ms (HIP events): the achievable HBM bandwidth, and a kernel whose
 * traffic is known (read `bytes`, write `bytes` per launch) to scale the
 * counters by.  Allocates and frees its buffers; bytes must be a positive
 * multiple of 16.
 */
int32_t h4d_stream_copy(int64_t bytes, int32_t reps, double *ms);

/*
 * Learned insertion proposal (every kind of handle: one box, a batch, or
 * speculative replicas; each box scores its own candidates with its own
 * Philox stream and trial index, and one matrix-core pass serves every box's
 * candidates).  A multiple-try form of
 * the uniform pair insertion of Eq. (4), exact for any network: a bias on
 * the initial flying-ion positions (the paper notes one would help and
 * leaves it out, Sec. II B 1) with the ratio corrected in the Rosenbluth
 * form of its distance bias (Sec. II B 4, Eqs. 15-16).  An insertion draws
 * k uniform candidate pair sites (Philox counters (trial, 4, j, 0 / 1)),
 * gives each the log weight lw = weight_scale * min(s, logit_cap), s the
 * network's logit of the site's 64 features on the state before the
 * trajectory, and flies the pair in at one chosen with probability
 * proportional to exp(lw) (uniform (trial, 5, 0, 0)); ln R of Eq. (6)
 * gains ln(W/k) - lw(chosen), W the sum of the weights.  A deletion weighs
 * the removed pair's site and k - 1 fresh candidates on the state after
 * its trajectory (pair removed) and ln R of Eq. (8) gains
 * lw(removed) - ln(W/k).  The factor is reported in h4d_trial.ln_proposal.
 *
 * Features of a site (31 per ion, then 2 for the pair), from the non-flying
 * atoms within rc = max cutoff, each pair term scaled by beta, clipped to
 * +-1e6 and summed in 64-bit fixed point (independent of atom order):
 *   0.1 x Gaussian shell counts of atom types 0..3 (six shells of width
 *   rc/6, centres (m + 1/2) rc/6, standard deviation rc/12, each term
 *   tapered by (1 - r^2/rc^2)^2 so the features are continuous); asinh of beta
 *   U_C, of beta |F_C|, of beta U_LJ at w = 0, of beta U_LJ and of beta
 *   exp(-kappa_sr w_max) U_C at w = w_max (Eq. 11); nearest-atom and
 *   nearest-counter-ion distances over rc (capped at 1); the pair's
 *   separation over rc (capped at 1) and asinh(beta u) of its own energy.
 *
 * The network: 64 -> 128 -> 128 -> 128 -> 1, GELU (tanh form) on the
 * hidden layers.  Parameters theta[41473] in the order W1[64][128], b1,
 * W2[128][128], b2, W3[128][128], b3, w4[128], b4 (W[i][o] maps input i to
 * output o).  Inference in the trial loop runs in BF16 on the matrix cores
 * with FP32 accumulation; training runs in FP32.  A network handle owns its
 * device memory; a system holding it (h4d_set_proposal) reads its
 * parameters at every trial, so it must outlive that use.
 */
typedef struct h4d_mlp h4d_mlp;

/* Network with Glorot-uniform weights from `seed`, zero biases. */
int32_t h4d_mlp_create(uint64_t seed, void *hip_stream, h4d_mlp **out);
int32_t h4d_mlp_destroy(h4d_mlp *net);
/* theta: 41473 host floats (the optimiser state is reset). */
int32_t h4d_mlp_set_weights(h4d_mlp *net, const float *theta);
int32_t h4d_mlp_get_weights(h4d_mlp *net, float *theta);
/* Logits of rows x 64 host features: bf16 = 1 the matrix-core inference
 * path, 0 the FP32 training forward. */
int32_t h4d_mlp_forward(h4d_mlp *net, int32_t rows, const float *features, int32_t bf16,
                        float *logits);
/*
 * The same logits without any allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  features (rows x 64) and logits (rows) are DEVICE pointers on
 * the device the network was created on (H4D_EINVAL if another device is
 * current); the kernels are enqueued on the network's stream and the call
 * returns without waiting (synchronise that stream before reading logits).
 * bf16 = 1: the matrix-core inference, reading features and writing logits
 * directly; bf16 = 0: the FP32 forward, its hidden activations in a static
 * workspace of the library (4 MiB per device, held until the process ends).
 * rows <= 4096, else H4D_EINVAL before any work.  The results equal
 * h4d_mlp_forward's bit for bit.  Calls that overlap on one device share the
 * workspace and race: serialise them (one stream, or events).
 */
int32_t h4d_mlp_forward_static(h4d_mlp *net, int32_t rows, const float *features, int32_t bf16,
                               float *logits);
/* Mean-squared loss of the FP32 logits against targets and its gradient
 * (grad[41473], host; may be NULL). */
int32_t h4d_mlp_loss_grad(h4d_mlp *net, int32_t rows, const float *features,
                          const float *targets, float *grad, float *loss);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr,
 * decoupled weight decay: theta -= lr * weight_decay * theta each step)
 * on minibatches of `batch` rows drawn from seeded shuffles of the data;
 * losses[steps] (host, may be NULL) receives each step's minibatch loss.
 * Training runs on standardized features (per-column mean and standard
 * deviation of the data); the affine map is folded into W1 and b1 before
 * return, so the network still reads raw features.  Each call starts a
 * fresh optimiser state.  Suggested target of a pilot insertion: its
 * clipped log ratio, clip(beta mu + I - beta dH, -100, 10). */
int32_t h4d_mlp_train(h4d_mlp *net, int32_t rows, const float *features, const float *targets,
                      int32_t steps, int32_t batch, float lr, float weight_decay, uint64_t seed,
                      float *losses);

/* Proposal of the following trials: k <= 0 the uniform proposal of Eq. (4);
 * k >= 1 the multiple-try proposal with k candidates, weighted by
 * exp(weight_scale * min(s, logit_cap)) with s the logit of `net` (NULL:
 * equal weights, which with k = 1 is the uniform proposal again and records
 * the features of every inserted or removed site).  The cap bounds how far
 * a network's extrapolation errors can steer the choice; weight_scale
 * (>= 0) tempers a network whose predictions are weak (0: the uniform
 * proposal).  Any cap and scale keep the method exact. */
int32_t h4d_set_proposal(h4d_system *sys, const h4d_mlp *net, int32_t k, double logit_cap,
                         double weight_scale);
/* Features of the last trial's inserted or removed pair site (64 floats; box 0). */
int32_t h4d_last_site_features(h4d_system *sys, float *out);
/* The last learned move's candidates: sites[6k], features[64k], logits[k]
 * (host, any may be NULL); returns k (>= 0) or an error.  Box 0, or box
 * `box` of a batch (a box with no learned move in its last trial keeps the
 * candidates of an earlier one). */
int32_t h4d_last_candidates(h4d_system *sys, int32_t cap, double *sites, float *features,
                            float *logits);
int32_t h4d_last_box_candidates(h4d_system *sys, int32_t box, int32_t cap, double *sites,
                                float *features, float *logits);
/* Test hook: features of n given sites (sites[6n]: cation xyz, anion xyz)
 * on the current state (no flying atoms). */
int32_t h4d_site_features(h4d_system *sys, int32_t n, const double *sites, float *features);

/* Release every resource of the handle. */
int32_t h4d_destroy(h4d_system *sys);

/* Message of the last failed call on this thread ("" if none). */
const char *h4d_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* H4D_H */
