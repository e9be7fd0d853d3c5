// h4d_kernels.hpp -- HIP kernels of H4D exchange trials on gfx950.
//
// One launch serves every box of a batch (a single system is a batch of
// one).  Box b owns atom slots [a0, a0 + cap) and cells [c0, c0 + nc) of the
// shared arrays, its own control block ctl[b] and trial record rec[b]; a
// block finds its box from the slot (or cell) it starts at.  All boxes run
// their current trial in lockstep rounds, each with its own N_f: a box whose
// trajectory has ended is frozen and its blocks return at once.
//
// Two copies of each box's configuration live in HBM:
//   canonical  cpos/ctag/ctype/cmol in ascending tag order: the state
//              between trials and the rollback snapshot during a trial;
//   working    the trial's atoms sorted by cell (spatial order) at its start:
//              pos[2] double4 (FP64 x, y, z + meta word), fx[2] uint4 (32-bit
//              fixed-point x, y, z + meta word), vel[2] double4, perm (working
//              -> canonical index), wmol.  pos/fx/vel ping-pong every step:
//              step k reads buffer k & 1, so a box's final state is in
//              buffer (N_f + 1) & 1.
// Verlet list: full list, blocked for wavefront-contiguous reads: atom slot
//   w's entry q sits at nbr[((w / A) * KQ + q / L) * 64 + (w % A) * L + q % L],
//   with L lanes per atom (4, 8 or 16), A = 64 / L atoms per wavefront,
//   KQ = cap_nbr / L.
// Every kernel reads the atom counts from the control blocks, so the launches
// of a round never wait on the host.
#pragma once
#include "h4d_device.hpp"

namespace h4d {

constexpr int kMaxLanes = 16;             // largest lanes-per-atom choice

struct Ctl {
    int n;            // atoms of the physical state
    int n_all;        // atoms including the two ghosts of an insertion
    int nsalt;
    int move;         // +1 insertion, -1 deletion, kMoveMD equilibrium phase, 0 nothing to do
    int ic, ia;       // slots of the flying cation / anion (canonical arrays)
    int wic, wia;     // their working slots
    int nf;           // NEMD steps of this trial
    int accepted;
    unsigned err;     // kErr* bits of this trial
    unsigned retry;   // 1: the trial must be recomputed
    int max_nbr, max_cell;
    int nfast[3];     // fast-atom list lengths (list k % 3 is read by step k)
    int max_fast;     // largest fast list of the trial
    int idle;         // 1: this box has run its quota of trials
    long long next_tag;
    long long trial;
    long long trial_end;   // the box idles once trial reaches this
    double u[8];
    double U0, K0, U1, K1;
    double Ulj, Uc, vir;
    double Wf[2];
    double Ufly0, Ufly1;   // U_fly(w_max) at the start / end state (FP64)
    double lnq;            // ln of the learned proposal's multiple-try factor (0: uniform)
    int instant;           // 1: the pair lies in V_ex, exchanged with no trajectory (nf = 0)
    long long md;          // equilibrium phases run (the phase's generator counter)
    long long md_end;      // the box idles in a phase round once md reaches this
};

// Trial record, same layout as h4d_trial of the C ABI.
struct TrialRec {
    int move, accepted, n_salt_before, n_salt_after, n_steps;
    unsigned flags;
    int n_atoms, n_rebuilds;
    long long trial, tag_c, tag_a;
    double dH, dU, dK, W_prot, E_switch, dM, ln_ratio, ln_u, ln_proposal, H0, H1;
};

constexpr unsigned kFlagEmpty = 1u, kFlagNonfinite = 2u, kFlagIdle = 8u, kFlagInstant = 16u;

struct KArgs {
    Geo G;
    const Box *box;
    const int *slot_box;      // box of atom slots [kBlock q, kBlock (q + 1))
    const int *cell_box;      // box of each cell
    int nbox;
    const PairCoef *coef;
    const double *mass;       // per type
    // canonical state
    double4 *cpos;
    double4 *cvel;            // the state's momenta (carried momenta, equilibrium phases)
    long long *ctag;
    int *ctype, *cmol;
    // working state
    double4 *pos[2];
    uint4 *fx[2];
    double4 *vel[2];
    int *perm, *wmol;
    uint4 *posb;              // fixed-point positions at the last list build
    double4 *force;           // test hook output (canonical slots)
    // compaction scratch (canonical order)
    double4 *tpos, *tvel;
    long long *ttag;
    int *ttype, *tmol;
    // lists
    int *nbr, *nnbr;
    int *cell_cnt[2], *cell_atoms[2], *cell_off;
    int *cell_sub[2];         // per cell: where each of its 8 sub-cells begins in its row
    int *slot_sub;            // sub-cell of each slot at its last binning
    int *fast;                // per box: 3 lists of kFastCap working slots
    int *molw;                // water atom (canonical 3m + q) -> working slot
    double4 *fw;              // forces on water atoms (working order)
    double *partial;          // per-block FP64 partial sums, 5 per block
    Ctl *ctl;                 // per box
    TrialRec *rec;            // per box
    int slots;                // atom slots of all boxes
    int step_blocks;          // blocks of the lanes-per-atom grids (the step
                              // grid adds one flyer block per box after them)
    int nbr_cap, cell_cap, ncell_total;
    int lanes, lanes_log2;    // lanes per atom in list traversals (4, 8 or 16)
    uint64_t seed;
    int n_steps, n_steps_min, n_steps_max;
    int md_steps;             // steps of an equilibrium phase
    int cation_type, anion_type;
};

// box of an atom slot / of a cell
__device__ __forceinline__ int box_of_slot(const KArgs &a, int slot) {
    return a.nbox == 1 ? 0 : a.slot_box[slot / kBlock];
}
__device__ __forceinline__ int box_of_cell(const KArgs &a, int cc) {
    return a.nbox == 1 ? 0 : a.cell_box[cc];
}

// working buffer of a kernel: b >= 0 as given, b < 0 the box's final buffer
__device__ __forceinline__ int buf_of(int b, const Ctl *c) { return b >= 0 ? b : ((c->nf + 1) & 1); }

// slot of entry q of atom slot w in the blocked list (L = a.lanes, A = 64 / L)
__device__ __forceinline__ size_t nbr_slot(const KArgs &a, int w, int q) {
    const int ll = a.lanes_log2, la = 6 - ll;
    return ((size_t)(w >> la) * (size_t)(a.nbr_cap >> ll) + (size_t)(q >> ll)) * kWave +
           (size_t)((w & ((1 << la) - 1)) << ll) + (size_t)(q & ((1 << ll) - 1));
}

// Coefficients are staged in LDS once per block.
struct CoefLds {
    PairCoef c[kMaxTypes * kMaxTypes];
};

__device__ __forceinline__ void load_coef(CoefLds &s, const PairCoef *g) {
    for (int q = threadIdx.x; q < kMaxTypes * kMaxTypes; q += blockDim.x) s.c[q] = g[q];
}

__device__ __forceinline__ uint4 fixed_of(const Box &B, double x, double y, double z, int meta) {
    return make_uint4(to_fixed(x, B.fx_inv[0]), to_fixed(y, B.fx_inv[1]), to_fixed(z, B.fx_inv[2]),
                      (unsigned)meta);
}

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
    int k = (int)(x / L * (double)nc);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// cell of a position, local to its box
__device__ __forceinline__ int cell_of(const Box &B, const double4 &p) {
    const int cx = cell_coord(p.x, B.L[0], B.ncell[0]);
    const int cy = cell_coord(p.y, B.L[1], B.ncell[1]);
    const int cz = cell_coord(p.z, B.L[2], B.ncell[2]);
    return (cz * B.ncell[1] + cy) * B.ncell[0] + cx;
}

// global index of the neighbour cell t (0..26, dz-major) of local cell (cx, cy, cz)
__device__ __forceinline__ int stencil_cell(const Box &B, int cx, int cy, int cz, int t) {
    const int nx = B.ncell[0], ny = B.ncell[1], nz = B.ncell[2];
    return B.c0 + (((cz + t / 9 - 1 + nz) % nz) * ny + (cy + (t / 3) % 3 - 1 + ny) % ny) * nx +
           (cx + t % 3 - 1 + nx) % nx;
}

// Sub-cell of a position: the octant of its cell (half a cell edge along
// each axis), bit d set for the upper half along axis d, from the same
// scaled coordinate as cell_coord.
__device__ __forceinline__ int subcell_of(const Box &B, const double4 &p) {
    const double x[3] = {p.x, p.y, p.z};
    int sub = 0;
    for (int d = 0; d < 3; ++d) {
        const double y = x[d] / B.L[d] * (double)B.ncell[d];
        int k = (int)y;
        k = k < 0 ? 0 : (k >= B.ncell[d] ? B.ncell[d] - 1 : k);
        int h = (int)(2.0 * y) - 2 * k;
        h = h < 0 ? 0 : (h > 1 ? 1 : h);
        sub |= h << d;
    }
    return sub;
}

// A position that is non-finite, or that the single periodic wrap of a step
// left outside the box (the atom moved more than a box edge in one step), is
// a trajectory that blew up: the atom is left out of the cells and the trial
// is marked non-finite (rejected, never recomputed).  The cells cannot fill
// up with such atoms, and every binned atom's fixed-point coordinate lies in
// its own cell, as the list build's padding entries assume.  (An edge value
// of exactly L is the rounding of a wrap from just below 0.)
__device__ __forceinline__ void bin_atom(const KArgs &a, const Box &B, Ctl *c, int cb, int w, const double4 &p) {
    if (!(p.x >= 0.0 && p.x <= B.L[0] && p.y >= 0.0 && p.y <= B.L[1] && p.z >= 0.0 && p.z <= B.L[2])) {
        atomicOr(&c->err, kErrNonfinite);
        return;
    }
    a.slot_sub[w] = B.use_cells ? subcell_of(B, p) : 0;
    const int cc = B.c0 + (B.use_cells ? cell_of(B, p) : 0);
    const int slot = atomicAdd(&a.cell_cnt[cb][cc], 1);
    if (slot < a.cell_cap) a.cell_atoms[cb][(size_t)cc * a.cell_cap + slot] = w;
    else { atomicOr(&c->err, kErrCell); atomicMax(&c->max_cell, slot + 1); }
}

// ==========================================================================
// Proposal on the canonical state, one block per box: move choice, ghost
// pair of an insertion, rank selection of a deletion (Eqs. 3-4; insertion
// or deletion with probability 1/2).  A box that has run its quota idles.
// ==========================================================================
// Bimodal bias (Sec. II B 4).  B_ins of Eq. (12) for an anion at pa and a
// cation at pc: V times the Eq. (14) density of the minimum-image offset
// along each edge.
__device__ __forceinline__ double bias_B(const KArgs &a, const Box &B, const double4 &pa, const double4 &pc) {
    const double al = a.G.bias_alpha, xb = a.G.bias_xb;
    const double d[3] = {min_image(pa.x - pc.x, B.L[0]), min_image(pa.y - pc.y, B.L[1]),
                         min_image(pa.z - pc.z, B.L[2])};
    double v = B.volume;
    for (int q = 0; q < 3; ++q)
        v *= B.bias_c[q] * (exp(-al * (d[q] - xb) * (d[q] - xb)) + exp(-al * (d[q] + xb) * (d[q] + xb)));
    return v;
}

// The insertion's anion offset along edge d: the Gaussian at -x_b or +x_b
// by one uniform, Box-Muller from it, redrawn (next attempt's counters)
// until it lies within half an edge -- a draw from Eq. (14).  The bias
// parameters are checked so that a redraw is all but never needed.
__device__ __forceinline__ double bias_offset(const KArgs &a, const Box &B, uint64_t t, int d) {
    const double half = 0.5 * B.L[d];
    const double sd = 1.0 / sqrt(2.0 * a.G.bias_alpha);
    double mu = a.G.bias_xb;
    for (int attempt = 0; attempt < 64; ++attempt) {
        const u64x4 r = philox(t, kPurposeBias, (uint64_t)(4 * attempt + d), 0, a.seed, B.stream);
        mu = unit_open(r.v[0]) < 0.5 ? -a.G.bias_xb : a.G.bias_xb;
        const double z = sqrt(-2.0 * log(unit_open(r.v[1]))) *
                         cos(6.283185307179586476925286766559 * unit_open(r.v[2]));
        const double x = mu + z * sd;
        if (fabs(x) <= half) return x;
    }
    return mu;
}

// A Maxwell-Boltzmann velocity (each component ~ N(0, kT/m), Sec. II A):
// Box-Muller normals of the stream (counter, purpose, tag), sd = sqrt(kT/m).
__device__ __forceinline__ double4 mb_velocity(const KArgs &a, const Box &B, uint64_t counter, uint64_t purpose,
                                               long long tag, double sd) {
    const double twopi = 6.283185307179586476925286766559;
    const u64x4 r = philox(counter, purpose, (uint64_t)tag, 0, a.seed, B.stream);
    const double u0 = unit_open(r.v[0]), u1 = unit_open(r.v[1]);
    const double u2 = unit_open(r.v[2]), u3 = unit_open(r.v[3]);
    const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
    return make_double4(sd * (r01 * cos(twopi * u1)), sd * (r01 * sin(twopi * u1)), sd * (r23 * cos(twopi * u3)),
                        0.0);
}

// Sign of the symmetric two-end momentum reversal of a trial with carried
// momenta: end 0 before the trajectory, end 1 after it, each -1 with
// probability 1/2.
__device__ __forceinline__ double reversal_sign(const KArgs &a, const Box &B, long long trial, int end) {
    const u64x4 r = philox((uint64_t)trial, kPurposeReverse, 0, 0, a.seed, B.stream);
    return unit_open(r.v[end]) < 0.5 ? -1.0 : 1.0;
}

// Equilibrium phase: the partly refreshed momenta of canonical atom i,
// c v + sqrt(1 - c^2) xi (generalized hybrid MC; c = 0 a full refresh).
__device__ __forceinline__ double4 refreshed_velocity(const KArgs &a, const Box &B, const Ctl *c, int i) {
    const double sd = sqrt(a.G.accel * a.G.kT / a.mass[a.ctype[i]]);
    const double4 xi = mb_velocity(a, B, (uint64_t)c->md, kPurposeRefresh, a.ctag[i], sd);
    const double4 v = a.cvel[i];
    const double cr = a.G.md_refresh, sr = sqrt(1.0 - cr * cr);
    return make_double4(cr * v.x + sr * xi.x, cr * v.y + sr * xi.y, cr * v.z + sr * xi.z, 0.0);
}

// Early rejection: does the anion lie inside the cube V_ex centred on the
// flying cation?  Such a pair is exchanged instantly (a conventional MC move
// with no trajectory), on insertion and deletion alike.
__device__ __forceinline__ bool in_ex_cube(const KArgs &a, const Box &B, const double4 &pc, const double4 &pa) {
    return fabs(min_image(pa.x - pc.x, B.L[0])) < a.G.v_ex_half && fabs(min_image(pa.y - pc.y, B.L[1])) < a.G.v_ex_half &&
           fabs(min_image(pa.z - pc.z, B.L[2])) < a.G.v_ex_half;
}

__global__ __launch_bounds__(kBlock) void k_propose(KArgs a, int force_move) {
    const int bi = blockIdx.x;
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    __shared__ int s_cnt[2][kBlock];
    __shared__ int s_move, s_kc, s_ka, s_ic, s_ia, s_n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const bool md = force_move == kMoveMD;
        int nf = a.n_steps;
        if (md) {   // equilibrium phase: the whole state in 3D, no flyers; u[7] its Metropolis uniform
            const u64x4 r0 = philox((uint64_t)c->md, kPurposeMD, 0, 0, a.seed, B.stream);
            for (int q = 0; q < 4; ++q) { c->u[q] = unit_open(r0.v[q]); c->u[4 + q] = 0.5; }
            c->u[7] = c->u[0];
            nf = a.md_steps;
        } else {
            const uint64_t t = (uint64_t)c->trial;
            const u64x4 r0 = philox(t, kPurposeSelect, 0, 0, a.seed, B.stream);
            const u64x4 r1 = philox(t, kPurposeSelect, 1, 0, a.seed, B.stream);
            for (int q = 0; q < 4; ++q) { c->u[q] = unit_open(r0.v[q]); c->u[4 + q] = unit_open(r1.v[q]); }
            if (a.n_steps_max > 0) {
                const u64x4 rn = philox(t, kPurposeNsteps, 0, 0, a.seed, B.stream);
                nf = a.n_steps_min + (int)floor(unit_open(rn.v[0]) * (double)(a.n_steps_max - a.n_steps_min + 1));
            }
        }
        c->nf = nf;
        c->idle = md ? c->md >= c->md_end : c->trial >= c->trial_end;
        int move = md ? kMoveMD : (force_move ? force_move : (c->u[0] < 0.5 ? 1 : -1));
        if ((move < 0 && c->nsalt == 0) || c->idle) move = 0;
        c->move = move;
        c->err = 0; c->retry = 0; c->accepted = 0;
        c->Wf[0] = c->Wf[1] = 0.0; c->Ufly0 = c->Ufly1 = 0.0;
        c->U0 = c->K0 = c->U1 = c->K1 = 0.0;
        c->lnq = 0.0;
        c->instant = 0;
        c->ic = c->ia = c->wic = c->wia = -1;
        c->nfast[0] = c->nfast[1] = c->nfast[2] = 0;
        c->max_fast = 0;
        c->n_all = c->n;
        s_move = move; s_n = c->n;
        s_kc = (int)floor(c->u[1] * (double)c->nsalt);
        s_ka = (int)floor(c->u[2] * (double)c->nsalt);
        s_ic = s_ia = -1;
        if (move == 1) {
            const int n = c->n;
            if (n + 2 > B.cap) {
                c->err |= kErrCap; c->retry = 1; c->move = 0; s_move = 0;
            } else {
                const int ic = B.a0 + n, ia = B.a0 + n + 1;
                const int tcat = a.cation_type, tan = a.anion_type;
                a.cpos[ic] = with_meta(wrap_coord(B.L[0] * c->u[1], B.L[0]),
                                       wrap_coord(B.L[1] * c->u[2], B.L[1]),
                                       wrap_coord(B.L[2] * c->u[3], B.L[2]), tcat | kFlyBit);
                if (a.G.bias_alpha > 0.0) {   // Sec. II B 4: offset from the cation drawn from Eq. (14)
                    const uint64_t t = (uint64_t)c->trial;
                    a.cpos[ia] = with_meta(wrap_coord(B.L[0] * c->u[1] + bias_offset(a, B, t, 0), B.L[0]),
                                           wrap_coord(B.L[1] * c->u[2] + bias_offset(a, B, t, 1), B.L[1]),
                                           wrap_coord(B.L[2] * c->u[3] + bias_offset(a, B, t, 2), B.L[2]),
                                           tan | kFlyBit);
                } else {
                    a.cpos[ia] = with_meta(wrap_coord(B.L[0] * c->u[4], B.L[0]),
                                           wrap_coord(B.L[1] * c->u[5], B.L[1]),
                                           wrap_coord(B.L[2] * c->u[6], B.L[2]), tan | kFlyBit);
                }
                a.ctag[ic] = c->next_tag; a.ctag[ia] = c->next_tag + 1;
                a.ctype[ic] = tcat; a.ctype[ia] = tan;
                a.cmol[ic] = -1; a.cmol[ia] = -1;
                c->ic = ic; c->ia = ia; c->n_all = n + 2;
                if (a.G.v_ex_half > 0.0 && in_ex_cube(a, B, a.cpos[ic], a.cpos[ia])) { c->nf = 0; c->instant = 1; }
            }
        }
    }
    __syncthreads();
    if (s_move >= 0) return;
    // deletion: the atom of each species with the drawn rank in tag order;
    // canonical order is tag order, so count species members per chunk and scan
    const int n = s_n;
    const int chunk = (n + kBlock - 1) / kBlock;
    const int lo = B.a0 + tid * chunk, hi = B.a0 + min(n, tid * chunk + chunk);
    int nc = 0, na = 0;
    for (int i = lo; i < hi; ++i) {
        const int ty = a.ctype[i];
        nc += (ty == a.cation_type);
        na += (ty == a.anion_type);
    }
    s_cnt[0][tid] = nc; s_cnt[1][tid] = na;
    __syncthreads();
    if (tid == 0) {
        int ac = 0, aa = 0;
        for (int q = 0; q < kBlock; ++q) {
            const int vc = s_cnt[0][q], va = s_cnt[1][q];
            s_cnt[0][q] = ac; s_cnt[1][q] = aa;
            ac += vc; aa += va;
        }
    }
    __syncthreads();
    const int pc = s_cnt[0][tid], pa = s_cnt[1][tid];
    if (s_kc >= pc && s_kc < pc + nc) {
        int r = pc;
        for (int i = lo; i < hi; ++i)
            if (a.ctype[i] == a.cation_type) { if (r == s_kc) { s_ic = i; break; } ++r; }
    }
    if (a.G.bias_alpha <= 0.0 && s_ka >= pa && s_ka < pa + na) {
        int r = pa;
        for (int i = lo; i < hi; ++i)
            if (a.ctype[i] == a.anion_type) { if (r == s_ka) { s_ia = i; break; } ++r; }
    }
    __syncthreads();
    if (a.G.bias_alpha > 0.0 && s_ic >= 0) {
        // Eq. (13): the anion with probability B_ins(r_a, r_c) / W, the first
        // in tag (canonical) order whose running sum exceeds u W; ln of
        // B_ins / B_del = W / (N + 1) for Eq. (16)
        __shared__ double s_w[kBlock];
        __shared__ double s_target;
        const double4 pc = a.cpos[s_ic];
        double part = 0.0;
        for (int i = lo; i < hi; ++i)
            if (a.ctype[i] == a.anion_type) part += bias_B(a, B, a.cpos[i], pc);
        s_w[tid] = part;
        __syncthreads();
        if (tid == 0) {
            double run = 0.0;
            for (int q = 0; q < kBlock; ++q) { const double v = s_w[q]; s_w[q] = run; run += v; }
            s_target = c->u[2] * run;
            c->lnq = log(run) - log((double)c->nsalt);
        }
        __syncthreads();
        const double start = s_w[tid], tg = s_target;
        if (tg >= start && tg < start + part) {
            double run = start;
            for (int i = lo; i < hi; ++i)
                if (a.ctype[i] == a.anion_type) {
                    run += bias_B(a, B, a.cpos[i], pc);
                    if (run > tg) { s_ia = i; break; }
                }
        }
        __syncthreads();
        if (tid == 0 && s_ia < 0) {   // rounding at the top end: the last anion
            for (int i = B.a0 + n - 1; i >= B.a0; --i)
                if (a.ctype[i] == a.anion_type) { s_ia = i; break; }
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int ic = s_ic, ia = s_ia;
        if (ic < 0 || ia < 0) {   // species counts disagree with nsalt: refuse the move
            c->err |= kErrCap; c->retry = 1; c->move = 0;
            return;
        }
        c->ic = ic; c->ia = ia;
        if (a.G.v_ex_half > 0.0 && in_ex_cube(a, B, a.cpos[ic], a.cpos[ia])) { c->nf = 0; c->instant = 1; }
        double4 p = a.cpos[ic];
        a.cpos[ic] = with_meta(p.x, p.y, p.z, meta_of(p) | kFlyBit);
        p = a.cpos[ia];
        a.cpos[ia] = with_meta(p.x, p.y, p.z, meta_of(p) | kFlyBit);
    }
}

// ==========================================================================
// Cells.  Binning uses atomics; each cell's members are then sorted by
// sub-cell and index so that every list is built in a fixed order (bitwise
// reproducible), and each sub-cell's members are contiguous.
// ==========================================================================
__global__ void k_cell_clear(KArgs a, int cb) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.ncell_total) a.cell_cnt[cb][q] = 0;
}

// bin the canonical atoms (trial start)
__global__ __launch_bounds__(kBlock) void k_bin_canonical(KArgs a, int cb) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (i - B.a0 >= c->n_all) return;
    bin_atom(a, B, c, cb, i, a.cpos[i]);
}

// bin the working atoms of every box with a trajectory, from its final buffer
__global__ __launch_bounds__(kBlock) void k_bin_working(KArgs a, int cb) {
    const int w = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, w);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (c->move == 0 || w - B.a0 >= c->n_all) return;
    bin_atom(a, B, c, cb, w, a.pos[buf_of(-1, c)][w]);
}

// One wavefront per cell: the members grouped by sub-cell (a counting pass,
// then each member's place in its group by the members of that group with a
// smaller index), so the order is (sub-cell, index) whatever order the
// binning atomics left.  Dynamic LDS: 3 cell_cap ints.
__global__ __launch_bounds__(kWave) void k_cell_sort(KArgs a, int cb) {
    extern __shared__ int buf[];
    int *sub = buf + a.cell_cap, *grp = sub + a.cell_cap;
    __shared__ int gstart[9], gfill[8];
    const int cc = blockIdx.x;
    const int cnt = min(a.cell_cnt[cb][cc], a.cell_cap);
    int *row = a.cell_atoms[cb] + (size_t)cc * a.cell_cap;
    if (threadIdx.x < 8) gfill[threadIdx.x] = 0;
    for (int q = threadIdx.x; q < cnt; q += kWave) {
        const int e = row[q];
        buf[q] = e;
        sub[q] = a.slot_sub[e];
    }
    __syncthreads();
    if (threadIdx.x < 8) {   // members of each sub-cell
        int r = 0;
        for (int p = 0; p < cnt; ++p) r += sub[p] == (int)threadIdx.x;
        gstart[threadIdx.x + 1] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        gstart[0] = 0;
        for (int q = 0; q < 8; ++q) gstart[q + 1] += gstart[q];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += kWave) {
        const int g = sub[q];
        grp[gstart[g] + atomicAdd(&gfill[g], 1)] = buf[q];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += kWave) {
        int g = 0;
        while (gstart[g + 1] <= q) ++g;
        const int e = grp[q];
        int r = gstart[g];
        for (int p = gstart[g]; p < gstart[g + 1]; ++p) r += grp[p] < e;
        row[r] = e;
    }
    if (threadIdx.x < 8) a.cell_sub[cb][8 * (size_t)cc + threadIdx.x] = gstart[threadIdx.x];
}

// exclusive scan of each box's cell counts (one block per box); cell_off
// holds the first working slot of every cell
__global__ __launch_bounds__(1024) void k_cell_scan(KArgs a, int cb) {
    __shared__ int part[1024];
    const Box &B = a.box[blockIdx.x];
    const int nc = B.nc;
    const int per = (nc + 1023) / 1024;
    const int lo = B.c0 + threadIdx.x * per, hi = B.c0 + min(nc, (int)threadIdx.x * per + per);
    int s = 0;
    for (int q = lo; q < hi; ++q) s += min(a.cell_cnt[cb][q], a.cell_cap);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = B.a0 + (threadIdx.x ? part[threadIdx.x - 1] : 0);
    for (int q = lo; q < hi; ++q) {
        a.cell_off[q] = run;
        run += min(a.cell_cnt[cb][q], a.cell_cap);
    }
}

// Trial start: gather the canonical atoms into cell order (working buffer 0),
// draw the Maxwell-Boltzmann momenta (keyed by tag, Box-Muller on Philox
// uniforms), and rewrite the cell rows with working slots.
__global__ __launch_bounds__(kWave) void k_gather_in(KArgs a, int cb) {
    const int cc = blockIdx.x;
    const int bi = box_of_cell(a, cc);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    const int cnt = min(a.cell_cnt[cb][cc], a.cell_cap);
    const int off = a.cell_off[cc];
    int *row = a.cell_atoms[cb] + (size_t)cc * a.cell_cap;
    const uint64_t t = (uint64_t)c->trial;
    for (int s = threadIdx.x; s < cnt; s += kWave) {
        const int src = row[s];
        const int w = off + s;
        const double4 p0 = a.cpos[src];
        const int mol = a.cmol[src];
        const int meta = meta_of(p0) | (mol >= 0 ? kMolBit : 0);
        const int ty = meta & kTypeMask;
        const double4 p = with_meta(p0.x, p0.y, p0.z, meta);
        a.pos[0][w] = p;
        if (mol >= 0) a.molw[src] = w;
        const uint4 q = fixed_of(B, p.x, p.y, p.z, meta);
        a.posb[w] = q;
        a.fx[0][w] = q;
        a.perm[w] = src;
        a.wmol[w] = mol;
        // momenta: an equilibrium phase's partial refresh of the carried
        // ones; with carried momenta a trial's start reversal of them (the
        // flyers' drawn afresh); else the trial's Maxwell-Boltzmann draw
        if (c->move == kMoveMD) {
            a.vel[0][w] = refreshed_velocity(a, B, c, src);
        } else if (a.G.momenta && !(meta & kFlyBit)) {
            const double s0 = reversal_sign(a, B, c->trial, 0);
            const double4 v = a.cvel[src];
            a.vel[0][w] = make_double4(s0 * v.x, s0 * v.y, s0 * v.z, 0.0);
        } else {
            a.vel[0][w] = mb_velocity(a, B, t, kPurposeMB, a.ctag[src], sqrt(a.G.accel * a.G.kT / a.mass[ty]));
        }
        if (src == c->ic) c->wic = w;
        if (src == c->ia) c->wia = w;
        row[s] = w;
    }
}

// Trial start, after the binning and the list build: a box whose cells or
// lists overflowed is recomputed with larger ones, and its trajectory this
// round is skipped (move 0).  A full cell leaves atoms out of the working
// buffer: a flyer among them has no working slot, and the slots past the
// gathered atoms hold no list.  A deletion's flags on the canonical pair are
// cleared here, as the rollback would.
__global__ void k_start_check(KArgs a) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= a.nbox) return;
    Ctl *c = a.ctl + bi;
    if (c->move == 0 || !(c->err & (kErrCell | kErrNbr))) return;
    if (c->move == -1) {
        double4 p = a.cpos[c->ic];
        a.cpos[c->ic] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
        p = a.cpos[c->ia];
        a.cpos[c->ia] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
    }
    c->move = 0;
}

// After a list build every atom is within the skin again: clear its fast flag.
__device__ __forceinline__ void unflag_fast(const KArgs &a, int b, int w, unsigned meta) {
    if (meta & kFastBit) {
        const unsigned m = meta & ~(unsigned)kFastBit;
        a.fx[b][w].w = m;
        double4 p = a.pos[b][w];
        a.pos[b][w] = with_meta(p.x, p.y, p.z, (int)m);
    }
}

// Which boxes a list build serves.  k = -1: every box (trial start, test
// hooks); k = -2: every box with a trajectory (end of trajectory); k >= 0:
// the rebuild before step k, for the boxes still running at step k.
__device__ __forceinline__ bool list_wanted(const Ctl *c, int k) {
    if (k == -1) return true;
    if (c->move == 0) return false;
    return k < 0 || k <= c->nf;
}

// ==========================================================================
// Verlet list (full, within r_list = max cutoff + skin), all-pairs form for
// boxes with fewer than 3 cells per edge: L lanes per atom test consecutive
// candidates; a ballot keeps the sequential order.
// ==========================================================================
__device__ __forceinline__ bool list_accepts(const KArgs &a, const Box &B, const uint4 &qi, int mi, int wi, int j,
                                             const uint4 &qj, int mj, float rl2) {
    if (j == wi) return false;
    if (mi >= 0 && mj == mi) return false;
    const float dx = (float)(int)(qi.x - qj.x) * B.fx_scale[0];
    const float dy = (float)(int)(qi.y - qj.y) * B.fx_scale[1];
    const float dz = (float)(int)(qi.z - qj.z) * B.fx_scale[2];
    return dx * dx + dy * dy + dz * dz < rl2;
}

__global__ __launch_bounds__(kBlock) void k_list_allpairs(KArgs a, int k, int b0, int cb) {
    const int slot0 = blockIdx.x * (kBlock >> a.lanes_log2);
    const int bi = box_of_slot(a, slot0);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (!list_wanted(c, k)) return;
    const int b = buf_of(b0, c);
    const int n_all = c->n_all;
    if (slot0 == B.a0 && threadIdx.x == 0) {
        a.cell_cnt[cb ^ 1][B.c0] = 0;
        c->nfast[0] = c->nfast[1] = c->nfast[2] = 0;
    }
    const int L = a.lanes;
    const int lane = threadIdx.x % kWave;
    const int s = lane & (L - 1);
    const int w = (blockIdx.x * kBlock + threadIdx.x) >> a.lanes_log2;
    if (w - B.a0 >= n_all) return;
    const uint4 qi = a.fx[b][w];
    const int mi = a.wmol[w];
    const float rl2 = (float)a.G.rlist2 * 1.00001f;     // superset margin for FP32 distances
    const int gshift = lane - s;
    const unsigned long long gmask = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
    const unsigned long long below = (1ull << s) - 1ull;
    int cnt = 0;
    for (int base = 0; base < n_all; base += L) {
        const int j = B.a0 + base + s;
        bool acc = false;
        if (base + s < n_all) acc = list_accepts(a, B, qi, mi, w, j, a.fx[b][j], a.wmol[j], rl2);
        const unsigned long long m = (__ballot(acc) >> gshift) & gmask;
        if (acc) {
            const int q = cnt + __popcll(m & below);
            if (q < a.nbr_cap) a.nbr[nbr_slot(a, w, q)] = j;
        }
        cnt += __popcll(m);
    }
    if (s == 0) {
        a.nnbr[w] = min(cnt, a.nbr_cap);
        a.posb[w] = qi;
        unflag_fast(a, b, w, qi.w);
        if (cnt > a.nbr_cap) { atomicOr(&c->err, kErrNbr); atomicMax(&c->max_nbr, cnt); }
    }
}

// Cell form with sub-cell culling.  A cell's row is ordered by sub-cell (its
// eight half-edge octants; cell_sub says where each begins), and `split`
// blocks of kListWaves wavefronts serve the centre atoms of one sub-cell
// (block s of the sub-cell takes its centre atoms t with (t / kListWaves) %
// split == s); with units = 1 they serve a whole cell instead, every range
// of the 27 cells staged (sparse cells, where a sub-cell would give the
// wavefronts too few centre atoms).  Cells have edge >= r_list, so along each axis the far half
// of a neighbouring cell lies at least one cell edge away from this
// sub-cell: of the 27 x 8 neighbouring sub-cells only the 5 x 5 x 5 around
// it can hold partners (125 / 216 of the 27 cells' volume), and only those
// ranges are read.  Of those, only the candidates within r_list of the
// centre sub-cell's box are kept in LDS (about half of them: the box grown
// by r_list is far smaller than the 5 x 5 x 5 block), as fixed-point
// coordinates + working slot in stencil order (cell, then sub-cell, then
// index), at most cand_cap at a time; each wavefront takes its centre atoms
// in turn and tests 64 candidates per ballot, two ballots per pass (the
// kept candidates are padded to whole pairs of wavefronts with entries that
// never match), appending partners in that order (a centre atom's running
// count stays in LDS when the kept candidates come in several batches).
// The lists are the same as without the box test.  MOL: rigid
// molecules present (pairs within a molecule are left out).  Dynamic LDS:
// (cand_cap + 128 + cell_cap) * 16 + cell_cap * 4 bytes.  Also records the build positions, clears this cell's count in the
// other buffer and the box's fast lists.
constexpr int kListWaves = 8;
constexpr int kSubRanges = 27 * 8;

template <bool C>
struct BoolTag {
    static constexpr bool value = C;
};

template <bool MOL>
__global__ __launch_bounds__(kListWaves * kWave) void k_list_cells(KArgs a, int k, int b0, int cb, int split,
                                                                    int cand_cap, int units) {
    extern __shared__ uint4 lds[];
    __shared__ int roff[kSubRanges + 1], rstart[kSubRanges], rcell[kSubRanges];
    __shared__ int s_c0, s_mc;
    const int cap = a.cell_cap;
    uint4 *cand = lds;                             // cand_cap + 128 staged candidates
    uint4 *ctr = lds + (size_t)cand_cap + 2 * kWave;   // the sub-cell's centre atoms (at most cap)
    int *ccount = reinterpret_cast<int *>(ctr + cap);
    // units 8: one centre sub-cell sc per block group; units 1: the whole cell (sc = -1)
    const int part = (int)blockIdx.x % split, un = ((int)blockIdx.x / split) % units;
    const int cc = (int)blockIdx.x / split / units, sc = units == 8 ? un : -1;
    const int bi = box_of_cell(a, cc);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (!list_wanted(c, k)) return;
    const int b = buf_of(b0, c);
    const int nx = B.ncell[0], ny = B.ncell[1], nz = B.ncell[2];
    const int lc = cc - B.c0;
    const int cx = lc % nx, cy = (lc / nx) % ny, cz = lc / (nx * ny);
    if (threadIdx.x < kSubRanges) {
        // range q: sub-cell q % 8 of stencil cell q / 8, kept when along every
        // axis it lies in the same cell or in the neighbour's near half, or
        // this sub-cell is the centre cell's half on the neighbour's side
        const int q = threadIdx.x, t = q >> 3, su = q & 7;
        auto keep = [](int d, int h, int hc) { return d == 0 || (d < 0 ? (h == 1 || hc == 0) : (h == 0 || hc == 1)); };
        const bool ok = sc < 0 || (keep(t % 3 - 1, su & 1, sc & 1) &&
                                   keep((t / 3) % 3 - 1, (su >> 1) & 1, (sc >> 1) & 1) &&
                                   keep(t / 9 - 1, (su >> 2) & 1, (sc >> 2) & 1));
        const int c2 = stencil_cell(B, cx, cy, cz, t);
        const int n2 = min(a.cell_cnt[cb][c2], cap);
        const int lo = min(a.cell_sub[cb][8 * (size_t)c2 + su], n2);
        const int hi = su < 7 ? min(a.cell_sub[cb][8 * (size_t)c2 + su + 1], n2) : n2;
        rcell[q] = c2;
        rstart[q] = lo;
        roff[q + 1] = ok ? max(0, hi - lo) : 0;
        // the centre cell is stencil entry 13
        if (t == 13 && sc >= 0 && su == sc) { s_c0 = lo; s_mc = max(0, hi - lo); }
        if (t == 13 && sc < 0 && su == 0) { s_c0 = 0; s_mc = n2; }
    }
    if (threadIdx.x == 0 && cc == B.c0 && part == 0 && un == 0) c->nfast[0] = c->nfast[1] = c->nfast[2] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        roff[0] = 0;
        for (int q = 0; q < kSubRanges; ++q) roff[q + 1] += roff[q];
    }
    __syncthreads();
    const int mc = s_mc;
    if (part * kListWaves >= mc) {               // no centre atoms for this block
        if (part == 0 && un == 0 && threadIdx.x == 0) a.cell_cnt[cb ^ 1][cc] = 0;
        return;
    }
    const int *crow = a.cell_atoms[cb] + (size_t)cc * cap + s_c0;
    for (int u = threadIdx.x; u < mc; u += blockDim.x) {
        const int j = crow[u];
        const uint4 q = a.fx[b][j];
        ctr[u] = make_uint4(q.x, q.y, q.z, (unsigned)j);
        ccount[u] = 0;
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const float rl2 = (float)a.G.rlist2 * 1.00001f;
    const float sx = B.fx_scale[0], sy = B.fx_scale[1], sz = B.fx_scale[2];
    const bool cubic = sx == sy && sy == sz;
    const unsigned lim = __float_as_uint(rl2) - 1u;
    uint4 far_pad;
    {
        auto opposite = [](int c, int n) {   // fixed-point coordinate of the cell centre, plus half the box
            return (unsigned)(((2.0 * c + 1.0) / (2.0 * n)) * 4294967296.0) + 0x80000000u;
        };
        far_pad = make_uint4(opposite(cx, nx), opposite(cy, ny), opposite(cz, nz), (unsigned)a.slots);
    }
    const float rl2u = (float)(a.G.rlist2 / ((double)sx * (double)sx)) * 1.00001f;   // in fixed-point units
    // the centre sub-cell's (or cell's) box in fixed-point units: its middle
    // and half its edge (plus a margin for the rounding of the binning), and
    // r_list^2 with a margin above the FP32 rounding of both distance tests
    uint3 mid;
    unsigned hw[3];
    {
        const int kc[3] = {cx, cy, cz};
        unsigned mv[3];
        for (int d = 0; d < 3; ++d) {
            const double n = (double)B.ncell[d];
            const double lo = sc < 0 ? kc[d] : kc[d] + 0.5 * ((sc >> d) & 1), half = sc < 0 ? 0.5 : 0.25;
            mv[d] = (unsigned)(unsigned long long)((lo + half) / n * 4294967296.0);
            hw[d] = (unsigned)(half / n * 4294967296.0) + 64u;
        }
        mid = make_uint3(mv[0], mv[1], mv[2]);
    }
    const float cull2 = (float)a.G.rlist2 * 1.0002f;
    auto near_box = [&](const uint4 &q) {
        auto gap = [](unsigned u, unsigned m, unsigned h) {
            const int d = (int)(u - m);
            const unsigned ad = d < 0 ? 0u - (unsigned)d : (unsigned)d;
            return (float)(ad > h ? ad - h : 0u);
        };
        const float gx = gap(q.x, mid.x, hw[0]) * sx, gy = gap(q.y, mid.y, hw[1]) * sy;
        const float gz = gap(q.z, mid.z, hw[2]) * sz;
        return gx * gx + gy * gy + gz * gz < cull2;
    };
    __shared__ int wkept[kListWaves];
    const unsigned lim_u = __float_as_uint(rl2u) - 1u;
    const int ll = a.lanes_log2;
    // The candidates within r_list of the centre unit's box (no centre atom
    // can pair with the others), in stencil order (cell, sub-cell, index),
    // are kept in LDS: staged in passes of one candidate per thread (its
    // range is the last whose offset does not exceed its position; empty
    // ranges share their offset), compacted by the waves' ballots and counts.
    // When the next pass might not fit, the kept candidates are scanned for
    // every centre atom first (a centre atom's running count stays in LDS).
    const int total = roff[kSubRanges];
    int kept = 0;
    auto flush = [&]() {
        // pad to whole pairs of wavefronts with entries that never match: the
        // null record's slot at the point opposite the centre cell's centre,
        // at least L/2 - h/2 >= h >= r_list from every centre atom along each
        // axis (3 or more cells per edge)
        if (threadIdx.x < 2 * kWave) cand[kept + threadIdx.x] = far_pad;
        __syncthreads();
        if (kept > 0) {
            for (int t = part * kListWaves + wave; t < mc; t += split * kListWaves) {
                // the centre atom is the same in every lane: scalar registers
                const uint4 qv = ctr[t];
                const unsigned qx = __builtin_amdgcn_readfirstlane(qv.x);
                const unsigned qy = __builtin_amdgcn_readfirstlane(qv.y);
                const unsigned qz = __builtin_amdgcn_readfirstlane(qv.z);
                const int wi = __builtin_amdgcn_readfirstlane((int)qv.w);
                const int mi = MOL ? a.wmol[wi] : -1;
                // the working slots of this atom's molecule (its partners in it
                // are left out), held in registers for the candidate loop
                int sib0 = -1, sib1 = -1, sib2 = -1;
                if (MOL && mi >= 0) {
                    const int c0 = B.a0 + 3 * mi;
                    sib0 = a.molw[c0]; sib1 = a.molw[c0 + 1]; sib2 = a.molw[c0 + 2];
                }
                int cnt = __builtin_amdgcn_readfirstlane(ccount[t]);
                char *dst = reinterpret_cast<char *>(a.nbr + nbr_slot(a, wi, 0));
                // entry q of the blocked list sits q + (q >> ll) (64 - L) entries in; a
                // list that overflows keeps rewriting its last entry (the build is
                // flagged and the trial recomputed with larger lists)
                const unsigned last = (unsigned)a.nbr_cap - 1u, gap = (unsigned)(kWave - (1 << ll));
                // a cubic box compares squared distances in fixed-point units
                // (three multiplies fewer per candidate)
                auto scan = [&](auto cubic_tag) {
                    constexpr bool CUBIC = decltype(cubic_tag)::value;
                    auto test = [&](const uint4 &qj) {
                        const int j = (int)qj.w;
                        float d2;
                        if constexpr (CUBIC) {
                            const float ux = (float)(int)(qx - qj.x);
                            const float uy = (float)(int)(qy - qj.y);
                            const float uz = (float)(int)(qz - qj.z);
                            d2 = ux * ux + uy * uy + uz * uz;
                        } else {
                            const float dx = (float)(int)(qx - qj.x) * sx;
                            const float dy = (float)(int)(qy - qj.y) * sy;
                            const float dz = (float)(int)(qz - qj.z) * sz;
                            d2 = dx * dx + dy * dy + dz * dz;
                        }
                        // 0 < d2 < r_list^2 as one unsigned compare of the float bits
                        // (monotonic for d2 >= 0); d2 = 0 is the atom itself
                        bool acc = __float_as_uint(d2) - 1u < (CUBIC ? lim_u : lim);
                        if (MOL) acc &= (j != sib0) & (j != sib1) & (j != sib2);   // ions carry no molecule (-1)
                        const unsigned long long msk = __builtin_amdgcn_ballot_w64(acc);
                        // the lane's entry: the running count plus the accepted lanes below it
                        const unsigned q = min(__builtin_amdgcn_mbcnt_hi((unsigned)(msk >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)msk, (unsigned)cnt)), last);
                        if (acc) *reinterpret_cast<int *>(dst + ((q + __umul24(q >> ll, gap)) << 2)) = j;
                        cnt += __popcll(msk);
                    };
                    // two wavefronts of candidates per pass, both read before either is tested
                    for (int base = 0; base < kept; base += 2 * kWave) {
                        const uint4 qa = cand[base + lane], qb = cand[base + kWave + lane];
                        test(qa);
                        test(qb);
                    }
                };
                if (cubic) scan(BoolTag<true>{});
                else scan(BoolTag<false>{});
                if (lane == 0) ccount[t] = cnt;
            }
        }
        __syncthreads();
        kept = 0;
    };
    for (int e0 = 0; e0 < total; e0 += (int)blockDim.x) {
        if (kept + min((int)blockDim.x, total - e0) > cand_cap) flush();
        const int e = e0 + (int)threadIdx.x;
        bool keep = false;
        uint4 rec = far_pad;
        if (e < total) {
            int lo = 0, hi = kSubRanges - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (roff[mid] <= e) lo = mid;
                else hi = mid - 1;
            }
            const int j = a.cell_atoms[cb][(size_t)rcell[lo] * cap + rstart[lo] + (e - roff[lo])];
            const uint4 q = a.fx[b][j];
            rec = make_uint4(q.x, q.y, q.z, (unsigned)j);
            keep = near_box(q);
        }
        const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
        if (lane == 0) wkept[wave] = __popcll(m);
        __syncthreads();
        int off = kept, all = kept;
        for (int v = 0; v < kListWaves; ++v) {
            off += v < wave ? wkept[v] : 0;
            all += wkept[v];
        }
        if (keep) cand[off + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = rec;
        kept = all;
        __syncthreads();
    }
    flush();
    for (int t = threadIdx.x; t < mc; t += blockDim.x) {
        if ((t / kListWaves) % split != part) continue;
        const uint4 qi = ctr[t];
        const int wi = (int)qi.w;
        const int cnt = ccount[t];
        a.nnbr[wi] = min(cnt, a.nbr_cap);
        a.posb[wi] = make_uint4(qi.x, qi.y, qi.z, a.fx[b][wi].w);
        unflag_fast(a, b, wi, a.fx[b][wi].w);
        if (cnt > a.nbr_cap) { atomicOr(&c->err, kErrNbr); atomicMax(&c->max_nbr, cnt); }
    }
    if (threadIdx.x == 0 && part == 0 && un == 0) a.cell_cnt[cb ^ 1][cc] = 0;
}

// Cell form for cells too large to stage in LDS: L lanes per atom walk the
// 27 stencil cells directly from global memory.
__global__ __launch_bounds__(kBlock) void k_list_lanes(KArgs a, int k, int b0, int cb) {
    const int P = kBlock >> a.lanes_log2;               // atoms per block
    const int slot0 = blockIdx.x * P;
    const int bi = box_of_slot(a, slot0);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (!list_wanted(c, k)) return;
    const int b = buf_of(b0, c);
    const int n_all = c->n_all;
    {   // this box's blocks clear its cells in the other buffer
        const int nblk = B.cap / P, lb = (slot0 - B.a0) / P;
        for (int q = lb * kBlock + threadIdx.x; q < B.nc; q += nblk * kBlock) a.cell_cnt[cb ^ 1][B.c0 + q] = 0;
        if (lb == 0 && threadIdx.x == 0) c->nfast[0] = c->nfast[1] = c->nfast[2] = 0;
    }
    const int L = a.lanes;
    const int lane = threadIdx.x % kWave;
    const int s = lane & (L - 1);
    const int w = (blockIdx.x * kBlock + threadIdx.x) >> a.lanes_log2;
    if (w - B.a0 >= n_all) return;
    const uint4 qi = a.fx[b][w];
    const int mi = a.wmol[w];
    const float rl2 = (float)a.G.rlist2 * 1.00001f;
    const int gshift = lane - s;
    const unsigned long long gmask = (1ull << L) - 1ull;
    const unsigned long long below = (1ull << s) - 1ull;
    const double4 pi = a.pos[b][w];
    const int cx = cell_coord(pi.x, B.L[0], B.ncell[0]);
    const int cy = cell_coord(pi.y, B.L[1], B.ncell[1]);
    const int cz = cell_coord(pi.z, B.L[2], B.ncell[2]);
    int cnt = 0;
    for (int t = 0; t < 27; ++t) {
        const int c2 = stencil_cell(B, cx, cy, cz, t);
        const int m = min(a.cell_cnt[cb][c2], a.cell_cap);
        const int *row = a.cell_atoms[cb] + (size_t)c2 * a.cell_cap;
        for (int base = 0; base < m; base += L) {
            const int u = base + s;
            bool acc = false;
            int j = 0;
            if (u < m) {
                j = row[u];
                acc = list_accepts(a, B, qi, mi, w, j, a.fx[b][j], a.wmol[j], rl2);
            }
            const unsigned long long mm = (__ballot(acc) >> gshift) & gmask;
            if (acc) {
                const int q = cnt + __popcll(mm & below);
                if (q < a.nbr_cap) a.nbr[nbr_slot(a, w, q)] = j;
            }
            cnt += __popcll(mm);
        }
    }
    if (s == 0) {
        a.nnbr[w] = min(cnt, a.nbr_cap);
        a.posb[w] = qi;
        unflag_fast(a, b, w, qi.w);
        if (cnt > a.nbr_cap) { atomicOr(&c->err, kErrNbr); atomicMax(&c->max_nbr, cnt); }
    }
}

// ==========================================================================
// Force on one atom at altitude w (flyers at w; with SP the anion flyer at
// w_ratio w, species-specific w_max), by the L lanes of its group,
// reduced over the group in a fixed order.  An atom that has moved beyond
// half the skin since the list build is "fast": pairs with fast atoms come
// from the fast list instead of the Verlet list, and a fast atom's own
// partners come from the 27 cells of the last build (cell edge >= r_c +
// skin covers every partner within r_c).  Every pair is counted once.
// ==========================================================================
// The block's FP32 force table for altitude wv and screening gscr (one
// entry per thread; call before a barrier): row ti, index tj | fly.  A flying
// partner sits at its own altitude (the anion's scaled by w_ratio with SP).
template <bool SP>
__device__ __forceinline__ void build_force_coef(const KArgs &a, ForceCoef *fcf, double wv, double gscr) {
    for (int q = threadIdx.x; q < kMaxTypes * kForceRow; q += blockDim.x) {
        const int ti = q / kForceRow, v = q % kForceRow, tj = v & kTypeMask;
        const bool fly = (v & kFlyBit) != 0;
        ForceCoef f = {0.0f, 0.0f, 0.0f, kFarW2};
        if (tj < kMaxTypes && !(v & kFastBit)) {
            const PairCoef &pc = a.coef[ti * kMaxTypes + tj];
            const float w2 = (float)(wv * wv);
            const float w2a = SP ? (float)((wv * a.G.w_ratio) * (wv * a.G.w_ratio)) : w2;
            const double sig6 = pc.sig2 * pc.sig2 * pc.sig2;
            f.lj12 = (float)(48.0 * pc.eps * sig6 * sig6);
            f.lj6 = (float)(24.0 * pc.eps * sig6);
            f.qqk = fly ? (float)gscr * pc.qqkf : pc.qqkf;
            f.w2 = fly ? ((SP && tj == a.anion_type) ? w2a : w2) : 0.0f;
        }
        fcf[q] = f;
    }
}

// NT: the list indices are loaded non-temporally (streamed past the caches),
// for lists too large to stay in the Infinity Cache between steps, where
// they would only evict the gathered records.
template <int PREC, int L, bool SP, bool NT = false>
__device__ __forceinline__ void group_force(const KArgs &a, const Box &B, const Ctl *c, const CoefLds &cf,
                                            const ForceCoef *fcf, int b, int cl, int w, int s, const double4 &pi,
                                            int mi, double wv, double gscr, const int *flist, int nfast, double &fx,
                                            double &fy, double &fz) {
    constexpr int A = kWave / L;
    const int ti = mi & kTypeMask;
    const bool own_fast = (mi & kFastBit) != 0;
    // molecule of this atom for the exclusions on the fast paths (the Verlet
    // list already leaves intramolecular pairs out)
    const int own_mol = (mi & kMolBit) ? a.wmol[w] : -1;
    auto same_mol = [&](int j) { return own_mol >= 0 && a.wmol[j] == own_mol; };
    const PairCoef *crow = cf.c + ti * kMaxTypes;
    if (PREC == 1) {
        const uint4 *F = a.fx[b];
        const uint4 qi = F[w];
        const ForceCoef *frow = fcf + ti * kForceRow;
        // displacements stay in fixed-point units (one scale per axis,
        // squared into the distance and applied to the summed force)
        const float sx2 = B.fx_scale[0] * B.fx_scale[0], sy2 = B.fx_scale[1] * B.fx_scale[1];
        const float sz2 = B.fx_scale[2] * B.fx_scale[2];
        float ax = 0.f, ay = 0.f, az = 0.f;
        // (an invalid entry may give a non-finite fs, e.g. a self pair at
        // s2 = 0: the select drops it)
        auto pair = [&](const uint4 &qj, bool valid) {
            const float ux = (float)(int)(qi.x - qj.x);
            const float uy = (float)(int)(qi.y - qj.y);
            const float uz = (float)(int)(qi.z - qj.z);
            const ForceCoef &fc = frow[(int)qj.w & (kTypeMask | kFlyBit)];
            const float s2 = fmaf(uz * sz2, uz, fmaf(uy * sy2, uy, fmaf(ux * sx2, ux, fc.w2)));
            const float fs = pair_fs_f32(a.G, fc, s2);
            const float f = valid ? fs : 0.0f;
            ax += f * ux; ay += f * uy; az += f * uz;
        };
        if (!own_fast) {
            // The Verlet list, in batches of NB neighbours (the list indices
            // of the next batch load while this batch's records are
            // gathered).  A fast partner and the null record that pads the
            // last batch index force-table entries that give exactly zero,
            // so no entry needs a validity test.
            constexpr int NB = 4;
            const int nn = a.nnbr[w];
            const int *base = a.nbr + ((size_t)(w / A) * (size_t)(a.nbr_cap / L)) * kWave + (size_t)(w % A) * L + s;
            const int nq = nn > s ? (nn - s + L - 1) / L : 0;
            const int null_slot = a.slots;
            auto index_at = [&](int q) {
                if constexpr (NT) return __builtin_nontemporal_load(base + (size_t)q * kWave);
                else return base[(size_t)q * kWave];
            };
            int jn[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) jn[u] = (u < nq) ? index_at(u) : null_slot;
            for (int k = 0; k < nq; k += NB) {
                int j[NB];
                uint4 q[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) j[u] = jn[u];
#pragma unroll
                for (int u = 0; u < NB; ++u) q[u] = F[j[u]];
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    jn[u] = (k + NB + u < nq) ? index_at(k + NB + u) : null_slot;
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const float ux = (float)(int)(qi.x - q[u].x);
                    const float uy = (float)(int)(qi.y - q[u].y);
                    const float uz = (float)(int)(qi.z - q[u].z);
                    const ForceCoef &fc = frow[(int)q[u].w & (kTypeMask | kFlyBit | kFastBit)];
                    const float s2 = fmaf(uz * sz2, uz, fmaf(uy * sy2, uy, fmaf(ux * sx2, ux, fc.w2)));
                    const float f = pair_fs_f32(a.G, fc, s2);
                    ax += f * ux; ay += f * uy; az += f * uz;
                }
            }
        } else if (!B.use_cells) {
            const int j1 = B.a0 + c->n_all;
            for (int j = B.a0 + s; j < j1; j += L) {
                const uint4 qj = F[j];
                pair(qj, j != w && !(qj.w & kFastBit) && !same_mol(j));
            }
        }
        // (cell form: a fast atom's pairs with the cells are summed by its
        // whole wavefront, fast_atoms_wave)
        for (int q = s; q < nfast; q += L) {
            const int j = flist[q];
            pair(F[j], j != w && !same_mol(j));
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            ax += __shfl_xor(ax, off, kWave);
            ay += __shfl_xor(ay, off, kWave);
            az += __shfl_xor(az, off, kWave);
        }
        fx = ax * B.fx_scale[0]; fy = ay * B.fx_scale[1]; fz = az * B.fx_scale[2];
    } else {
        const double4 *P = a.pos[b];
        double ax = 0.0, ay = 0.0, az = 0.0;
        const double w2 = wv * wv;
        const double w2a = SP ? (wv * a.G.w_ratio) * (wv * a.G.w_ratio) : w2;
        auto pair = [&](const double4 &pj, bool valid) {
            if (!valid) return;
            const double dx = min_image(pi.x - pj.x, B.L[0]);
            const double dy = min_image(pi.y - pj.y, B.L[1]);
            const double dz = min_image(pi.z - pj.z, B.L[2]);
            const int mj = meta_of(pj);
            const bool fj = (mj & kFlyBit) != 0;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double s2 = fj ? r2 + ((SP && (mj & kTypeMask) == a.anion_type) ? w2a : w2) : r2;
            if (s2 < a.G.rc_max2) {
                const double fs = pair_fs_f64(a.G, crow[mj & kTypeMask], s2, fj ? gscr : 1.0);
                ax += fs * dx; ay += fs * dy; az += fs * dz;
            }
        };
        if (!own_fast) {
            const int nn = a.nnbr[w];
            const int *base = a.nbr + ((size_t)(w / A) * (size_t)(a.nbr_cap / L)) * kWave + (size_t)(w % A) * L + s;
            for (int q = s, k = 0; q < nn; q += L, ++k) {
                const double4 pj = P[base[(size_t)k * kWave]];
                pair(pj, !(meta_of(pj) & kFastBit));
            }
        } else if (B.use_cells) {
            const int cx = cell_coord(pi.x, B.L[0], B.ncell[0]);
            const int cy = cell_coord(pi.y, B.L[1], B.ncell[1]);
            const int cz = cell_coord(pi.z, B.L[2], B.ncell[2]);
            for (int t = 0; t < 27; ++t) {
                const int c2 = stencil_cell(B, cx, cy, cz, t);
                const int m = min(a.cell_cnt[cl][c2], a.cell_cap);
                const int *row = a.cell_atoms[cl] + (size_t)c2 * a.cell_cap;
                for (int u = s; u < m; u += L) {
                    const int j = row[u];
                    const double4 pj = P[j];
                    pair(pj, j != w && !(meta_of(pj) & kFastBit) && !same_mol(j));
                }
            }
        } else {
            const int j1 = B.a0 + c->n_all;
            for (int j = B.a0 + s; j < j1; j += L) {
                const double4 pj = P[j];
                pair(pj, j != w && !(meta_of(pj) & kFastBit) && !same_mol(j));
            }
        }
        for (int q = s; q < nfast; q += L) {
            const int j = flist[q];
            pair(P[j], j != w && !same_mol(j));
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            ax += __shfl_xor(ax, off, kWave);
            ay += __shfl_xor(ay, off, kWave);
            az += __shfl_xor(az, off, kWave);
        }
        fx = ax; fy = ay; fz = az;
    }
}

// FP32 forces on the fast atoms of one wavefront from the 27 cells of the
// last build (cell form): each fast atom in turn, lowest lane first, with
// all 64 lanes sharing its candidates (an atom's own L lanes would take
// 64 / L times as long and hold up the kernel).  Pairs with other fast atoms
// come from the fast list in group_force.  Every lane of the wavefront
// calls this; mine marks lane s = 0 of a fast, non-flying, active atom, and
// that lane's force gains the sum (fixed butterfly order).
template <bool SP>
__device__ __forceinline__ void fast_atoms_wave(const KArgs &a, const Box &B, const ForceCoef *fcf, int b, int cl,
                                                bool mine, int w, int lane, double wv, double gscr, double &fx,
                                                double &fy, double &fz) {
    unsigned long long fm = __ballot(mine);
    if (fm == 0ull || !B.use_cells) return;
    const uint4 *F = a.fx[b];
    const float sx = B.fx_scale[0], sy = B.fx_scale[1], sz = B.fx_scale[2];
    while (fm != 0ull) {
        const int src = __ffsll((long long)fm) - 1;
        fm &= fm - 1ull;
        const int wf = __shfl(w, src, kWave);
        const uint4 qi = F[wf];
        const double4 pf = a.pos[b][wf];
        const int mi = (int)qi.w;
        const ForceCoef *frow = fcf + (mi & kTypeMask) * kForceRow;
        const int own_mol = (mi & kMolBit) ? a.wmol[wf] : -1;
        const int cx = cell_coord(pf.x, B.L[0], B.ncell[0]);
        const int cy = cell_coord(pf.y, B.L[1], B.ncell[1]);
        const int cz = cell_coord(pf.z, B.L[2], B.ncell[2]);
        float ax = 0.f, ay = 0.f, az = 0.f;
        for (int t = 0; t < 27; ++t) {
            const int c2 = stencil_cell(B, cx, cy, cz, t);
            const int m = min(a.cell_cnt[cl][c2], a.cell_cap);
            const int *row = a.cell_atoms[cl] + (size_t)c2 * a.cell_cap;
            for (int u = lane; u < m; u += kWave) {
                const int j = row[u];
                const uint4 qj = F[j];
                const bool valid = j != wf && !(qj.w & kFastBit) && !(own_mol >= 0 && a.wmol[j] == own_mol);
                const float dx = (float)(int)(qi.x - qj.x) * sx;
                const float dy = (float)(int)(qi.y - qj.y) * sy;
                const float dz = (float)(int)(qi.z - qj.z) * sz;
                const ForceCoef &fc = frow[(int)qj.w & (kTypeMask | kFlyBit)];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float fs = pair_fs_f32(a.G, fc, r2 + fc.w2);
                const float f = valid ? fs : 0.0f;
                ax += f * dx; ay += f * dy; az += f * dz;
            }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            ax += __shfl_xor(ax, off, kWave);
            ay += __shfl_xor(ay, off, kWave);
            az += __shfl_xor(az, off, kWave);
        }
        if (lane == src) { fx += ax; fy += ay; fz += az; }
    }
}

// Displacement since the last list build, from the fixed-point coordinates
// (flagged slightly early: the threshold is lowered by 1e-5 relative).
__device__ __forceinline__ bool moved_beyond_half_skin(const KArgs &a, const Box &B, const uint4 &q, const uint4 &qb) {
    const float dx = (float)(int)(q.x - qb.x) * B.fx_scale[0];
    const float dy = (float)(int)(q.y - qb.y) * B.fx_scale[1];
    const float dz = (float)(int)(q.z - qb.z) * B.fx_scale[2];
    return dx * dx + dy * dy + dz * dz > (float)a.G.half_skin2 * 0.99999f;
}

// --------------------------------------------------------------------------
// Flying work of one flyer at x_k (one wavefront per flyer): the trapezoid
// share 1/2 [U_fly(x_k; w_{k+1}) - U_fly(x_k; w_{k-1})] (endpoints clamped),
// accumulated in FP64 (pair energies in the precision of the pass).  With
// SP (species-specific w_max) each flyer sits at its own altitude, the
// screening follows the flyers' mean altitude, and the flyer-flyer pair,
// whose altitude difference now changes, adds its share once (wave 0).
// --------------------------------------------------------------------------
template <int PREC, bool SP>
__device__ void flyer_work(const KArgs &a, const Box &B, Ctl *c, const CoefLds &cf, int b, int k, const int *flist,
                           int nfast) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (wave > 1) return;
    const int move = c->move, nf = c->nf;
    if (move == 0 || move == kMoveMD || k > nf) return;
    const int f = wave == 0 ? c->wic : c->wia;
    const int other = wave == 0 ? c->wia : c->wic;
    if (f < 0 || other < 0) return;   // a flyer with no working slot (its trial is not kept)
    const double wlo0 = altitude(a.G, move, k > 0 ? k - 1 : 0, nf);
    const double whi0 = altitude(a.G, move, k < nf ? k + 1 : nf, nf);
    // this flyer's own altitudes (wave 1 is the anion) and the screening altitudes
    const double rf = (SP && wave == 1) ? a.G.w_ratio : 1.0;
    const double wlo = wlo0 * rf, whi = whi0 * rf;
    const double slo = SP ? 0.5 * wlo0 * (1.0 + a.G.w_ratio) : wlo0;
    const double shi = SP ? 0.5 * whi0 * (1.0 + a.G.w_ratio) : whi0;
    const double dflo = SP ? wlo0 * (1.0 - a.G.w_ratio) : 0.0, dfhi = SP ? whi0 * (1.0 - a.G.w_ratio) : 0.0;
    double dsum = 0.0;
    const int nn = a.nnbr[f];
    // the flyer's list (partners that are now fast are taken from the fast list)
    const int ntot = nn + nfast;
    if (PREC == 1) {
        const uint4 qf = a.fx[b][f];
        const int tf = (int)qf.w & kTypeMask;
        const float wl2 = (float)(wlo * wlo), wh2 = (float)(whi * whi);
        const float glo = (float)exp(-a.G.kappa * slo), ghi = (float)exp(-a.G.kappa * shi);
        if (SP && wave == 0 && lane == 0) {   // the flyer-flyer pair, unscreened
            const uint4 qo = a.fx[b][other];
            const float dx = (float)(int)(qf.x - qo.x) * B.fx_scale[0];
            const float dy = (float)(int)(qf.y - qo.y) * B.fx_scale[1];
            const float dz = (float)(int)(qf.z - qo.z) * B.fx_scale[2];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const PairCoef &cc = cf.c[tf * kMaxTypes + ((int)qo.w & kTypeMask)];
            const float sl = r2 + (float)(dflo * dflo), sh = r2 + (float)(dfhi * dfhi);
            const float ulo = sl < a.G.rc_max2f ? pair_u_f32(a.G, cc, sl, 1.0f) : 0.0f;
            const float uhi = sh < a.G.rc_max2f ? pair_u_f32(a.G, cc, sh, 1.0f) : 0.0f;
            dsum += (double)uhi - (double)ulo;
        }
        for (int q = lane; q < ntot; q += kWave) {
            const int j = q < nn ? a.nbr[nbr_slot(a, f, q)] : flist[q - nn];
            if (j == other) continue;
            const uint4 qj = a.fx[b][j];
            if (q < nn && (qj.w & kFastBit)) continue;
            const float dx = (float)(int)(qf.x - qj.x) * B.fx_scale[0];
            const float dy = (float)(int)(qf.y - qj.y) * B.fx_scale[1];
            const float dz = (float)(int)(qf.z - qj.z) * B.fx_scale[2];
            const float r2 = dx * dx + dy * dy + dz * dz;
            const PairCoef &cc = cf.c[tf * kMaxTypes + ((int)qj.w & kTypeMask)];
            const float ulo = (r2 + wl2 < a.G.rc_max2f) ? pair_u_f32(a.G, cc, r2 + wl2, glo) : 0.0f;
            const float uhi = (r2 + wh2 < a.G.rc_max2f) ? pair_u_f32(a.G, cc, r2 + wh2, ghi) : 0.0f;
            dsum += (double)uhi - (double)ulo;
        }
    } else {
        const double4 *P = a.pos[b];
        const double4 pf = P[f];
        const int tf = meta_of(pf) & kTypeMask;
        const double glo = exp(-a.G.kappa * slo), ghi = exp(-a.G.kappa * shi);
        if (SP && wave == 0 && lane == 0) {   // the flyer-flyer pair, unscreened
            const double4 po = P[other];
            const double dx = min_image(pf.x - po.x, B.L[0]);
            const double dy = min_image(pf.y - po.y, B.L[1]);
            const double dz = min_image(pf.z - po.z, B.L[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const PairCoef &cc = cf.c[tf * kMaxTypes + (meta_of(po) & kTypeMask)];
            double ulj, uc, fs, ulo = 0.0, uhi = 0.0;
            if (r2 + dflo * dflo < a.G.rc_max2) { pair_u_f64(a.G, cc, r2 + dflo * dflo, 1.0, ulj, uc, fs); ulo = ulj + uc; }
            if (r2 + dfhi * dfhi < a.G.rc_max2) { pair_u_f64(a.G, cc, r2 + dfhi * dfhi, 1.0, ulj, uc, fs); uhi = ulj + uc; }
            dsum += uhi - ulo;
        }
        for (int q = lane; q < ntot; q += kWave) {
            const int j = q < nn ? a.nbr[nbr_slot(a, f, q)] : flist[q - nn];
            if (j == other) continue;
            const double4 pj = P[j];
            if (q < nn && (meta_of(pj) & kFastBit)) continue;
            const double dx = min_image(pf.x - pj.x, B.L[0]);
            const double dy = min_image(pf.y - pj.y, B.L[1]);
            const double dz = min_image(pf.z - pj.z, B.L[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const PairCoef &cc = cf.c[tf * kMaxTypes + (meta_of(pj) & kTypeMask)];
            double ulj, uc, fs, ulo = 0.0, uhi = 0.0;
            if (r2 + wlo * wlo < a.G.rc_max2) { pair_u_f64(a.G, cc, r2 + wlo * wlo, glo, ulj, uc, fs); ulo = ulj + uc; }
            if (r2 + whi * whi < a.G.rc_max2) { pair_u_f64(a.G, cc, r2 + whi * whi, ghi, ulj, uc, fs); uhi = ulj + uc; }
            dsum += uhi - ulo;
        }
    }
    dsum = wave_sum(dsum);
    if (lane == 0) c->Wf[wave] += 0.5 * dsum;
}

// ==========================================================================
// One NEMD step k (k = 0..nf), fused: F(x_k; w_k) from the list (L lanes per
// atom); the second half kick of step k-1 (k > 0); the first half kick and
// drift of step k (k < nf) into the other buffer.  Flyers stay fixed in 3D.
// bin != 0: also bin the new positions for the rebuild before step k+1.
// Blocks [0, step_blocks) cover the atom slots; block step_blocks + b
// evaluates the flying work of box b.
// ==========================================================================
template <int PREC, int L, bool SP, bool NT>
__global__ __launch_bounds__(kBlock) void k_step(KArgs a, int k, int b, int bin, int cl) {
    const bool flyer_block = (int)blockIdx.x >= a.step_blocks;
    const int slot0 = (int)blockIdx.x * (kBlock / L);
    const int bi = flyer_block ? (int)blockIdx.x - a.step_blocks : box_of_slot(a, slot0);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    const int move = c->move, nf = c->nf, n_all = c->n_all;
    if (move == 0 || k > nf) return;
    if (!flyer_block && slot0 - B.a0 >= n_all) return;
    __shared__ CoefLds cf;
    load_coef(cf, a.coef);
    const double wv = altitude(a.G, move, k, nf);
    // Eq. 11 screening at the flyers' mean altitude
    const double gscr = exp(-a.G.kappa * (SP ? 0.5 * wv * (1.0 + a.G.w_ratio) : wv));
    __shared__ ForceCoef fcf[PREC == 1 ? kMaxTypes * kForceRow : 1];
    if (PREC == 1) build_force_coef<SP>(a, fcf, wv, gscr);
    const int lr = k % 3, lw = (k + 1) % 3;       // fast list read / written by this step
    const int nfast = min(c->nfast[lr], kFastCap);
    int *fast = a.fast + (size_t)bi * 3 * kFastCap;
    // the list was appended to in atomic order: sort it (fixed summation order)
    __shared__ int sfast_in[kFastCap], sfast[kFastCap];
    if (nfast > 0) {
        for (int q = threadIdx.x; q < nfast; q += kBlock) sfast_in[q] = fast[lr * kFastCap + q];
        __syncthreads();
        for (int q = threadIdx.x; q < nfast; q += kBlock) {
            const int e = sfast_in[q];
            int r = 0;
            for (int p = 0; p < nfast; ++p) r += (sfast_in[p] < e);
            sfast[r] = e;
        }
    }
    __syncthreads();
    const int *flist = sfast;
    if (flyer_block) {
        if (threadIdx.x == 0) c->nfast[(k + 2) % 3] = 0;
        flyer_work<PREC, SP>(a, B, c, cf, b, k, flist, nfast);
        return;
    }
    const int lane = threadIdx.x % kWave;
    const int s = lane % L;
    const int w = slot0 + (int)threadIdx.x / L;
    const bool act = w - B.a0 < n_all;
    const int wc = act ? w : B.a0;
    const double4 pi = a.pos[b][wc];
    const int mi = meta_of(pi);
    const bool fly = (mi & kFlyBit) != 0;
    const int ti = mi & kTypeMask;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (act && !fly)
        group_force<PREC, L, SP, NT>(a, B, c, cf, fcf, b, cl, wc, s, pi, mi, wv, gscr, flist, nfast, fx, fy, fz);
    if (PREC == 1) fast_atoms_wave<SP>(a, B, fcf, b, cl, act && !fly && s == 0 && (mi & kFastBit), wc, lane, wv, gscr,
                                       fx, fy, fz);
    if (!act || s != 0) return;
    if (mi & kMolBit) {   // rigid water: integrated by k_settle
        a.fw[wc] = make_double4(fx, fy, fz, 0.0);
        return;
    }
    double4 v = a.vel[b][wc];
    double x = pi.x, y = pi.y, z = pi.z;
    int mo = mi;
    if (!fly) {
        const double hm = a.G.half_dt * a.G.accel / a.mass[ti];
        if (k > 0) { v.x += hm * fx; v.y += hm * fy; v.z += hm * fz; }
        if (k < nf) {
            v.x += hm * fx; v.y += hm * fy; v.z += hm * fz;
            x = wrap_coord(pi.x + a.G.dt * v.x, B.L[0]);
            y = wrap_coord(pi.y + a.G.dt * v.y, B.L[1]);
            z = wrap_coord(pi.z + a.G.dt * v.z, B.L[2]);
        }
    }
    uint4 qn = fixed_of(B, x, y, z, mi);
    if (!fly && (mo & kFastBit) == 0 && moved_beyond_half_skin(a, B, qn, a.posb[wc])) mo |= kFastBit;
    if (mo & kFastBit) {   // (re-)register in the list read by the next step
        const int slot = atomicAdd(&c->nfast[lw], 1);
        if (slot < kFastCap) fast[lw * kFastCap + slot] = wc;
        else atomicOr(&c->err, kErrFast);
        atomicMax(&c->max_fast, slot + 1);
    }
    qn.w = (unsigned)mo;
    const double4 pn = with_meta(x, y, z, mo);
    a.pos[b ^ 1][wc] = pn;
    a.vel[b ^ 1][wc] = v;
    a.fx[b ^ 1][wc] = qn;
    if (bin && k < nf) bin_atom(a, B, c, cl ^ 1, wc, pn);
}

// Test hook: forces of the working buffer-0 state with the flags it carries;
// written at the canonical slots.
template <int PREC, int L, bool SP>
__global__ __launch_bounds__(kBlock) void k_forces(KArgs a, double wv) {
    const int slot0 = (int)blockIdx.x * (kBlock / L);
    const int bi = box_of_slot(a, slot0);
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    __shared__ CoefLds cf;
    load_coef(cf, a.coef);
    const double gscr = exp(-a.G.kappa * (SP ? 0.5 * wv * (1.0 + a.G.w_ratio) : wv));
    __shared__ ForceCoef fcf[PREC == 1 ? kMaxTypes * kForceRow : 1];
    if (PREC == 1) build_force_coef<SP>(a, fcf, wv, gscr);
    __syncthreads();
    const int lane = threadIdx.x % kWave;
    const int s = lane % L;
    const int w = slot0 + (int)threadIdx.x / L;
    const bool act = w - B.a0 < c->n_all;
    const int wc = act ? w : B.a0;
    const double4 pi = a.pos[0][wc];
    const int mi = meta_of(pi);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (act && !(mi & kFlyBit))
        group_force<PREC, L, SP>(a, B, c, cf, fcf, 0, 0, wc, s, pi, mi, wv, gscr, a.fast, 0, fx, fy, fz);
    if (PREC == 1) fast_atoms_wave<SP>(a, B, fcf, 0, 0, act && !(mi & kFlyBit) && s == 0 && (mi & kFastBit), wc,
                                       lane, wv, gscr, fx, fy, fz);
    if (act && s == 0) a.force[a.perm[wc]] = make_double4(fx, fy, fz, 0.0);
}

// ==========================================================================
// FP64 energies.  mode 0: flyers at altitude w (NEMD); mode 1: every pair
// with a flyer left out.  mode -1: chosen from the move (start: insertion
// excludes its ghosts; end: deletion excludes the removed pair; else all
// atoms at w = 0).  Each pair is counted half from each side.
// which: 0 start of trial, 1 end, 2 observables / test hook (every box).
// b < 0: each box's final buffer.
// ==========================================================================
__global__ __launch_bounds__(kBlock) void k_energy(KArgs a, int which, int mode, double wv, int b0) {
    __shared__ CoefLds cf;
    __shared__ double red[5][kBlock / kWave];
    const int slot0 = (int)blockIdx.x * (kBlock >> a.lanes_log2);
    const int bi = box_of_slot(a, slot0);
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    load_coef(cf, a.coef);
    __syncthreads();
    const int move = c->move;
    const bool skip = which < 2 && move == 0;
    if (mode < 0) mode = ((which == 0 && move == 1) || (which == 1 && move == -1)) ? 1 : 0;
    const int b = buf_of(b0, c);
    const int lane = threadIdx.x % kWave;
    const int s = lane & (a.lanes - 1);
    const int w = (blockIdx.x * kBlock + threadIdx.x) >> a.lanes_log2;
    double ulj_s = 0.0, uc_s = 0.0, k_s = 0.0, vir_s = 0.0, fly_s = 0.0;
    if (!skip && w - B.a0 < c->n_all) {
        const double4 *P = a.pos[b];
        const double4 pi = P[w];
        const int mi = meta_of(pi);
        const bool fi = (mi & kFlyBit) != 0;
        const int ti = mi & kTypeMask;
        // species-specific w_max: each flyer at its own factor times the
        // cation's altitude, screening at the flyers' mean altitude
        const double ri = (ti == a.anion_type) ? a.G.w_ratio : 1.0;
        const double gs = exp(-a.G.kappa * (0.5 * wv * (1.0 + a.G.w_ratio)));
        const double gmax = exp(-a.G.kappa * (0.5 * a.G.w_max * (1.0 + a.G.w_ratio)));
        const double wmax_i = a.G.w_max * ri;
        const int nn = a.nnbr[w];
        for (int q = s; q < nn; q += a.lanes) {
            const int j = a.nbr[nbr_slot(a, w, q)];
            const double4 pj = P[j];
            const int mj = meta_of(pj);
            const bool fj = (mj & kFlyBit) != 0;
            const double dx = min_image(pi.x - pj.x, B.L[0]);
            const double dy = min_image(pi.y - pj.y, B.L[1]);
            const double dz = min_image(pi.z - pj.z, B.L[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const PairCoef &cc = cf.c[ti * kMaxTypes + (mj & kTypeMask)];
            double ulj, uc, fs;
            // switch energy U_fly(w_max), counted from the flyer's side:
            // flyer-nonflyer at the 4D distance, flyer-flyer half from each
            const double rj = ((mj & kTypeMask) == a.anion_type) ? a.G.w_ratio : 1.0;
            if (fi && which < 2) {
                const double dmax = wmax_i - a.G.w_max * rj;
                if (!fj && r2 + wmax_i * wmax_i < a.G.rc_max2) {
                    pair_u_f64(a.G, cc, r2 + wmax_i * wmax_i, gmax, ulj, uc, fs);
                    fly_s += ulj + uc;
                } else if (fj && r2 + dmax * dmax < a.G.rc_max2) {
                    pair_u_f64(a.G, cc, r2 + dmax * dmax, 1.0, ulj, uc, fs);
                    fly_s += 0.5 * (ulj + uc);
                }
            }
            if (mode == 1 && (fi || fj)) continue;
            const double wi = (mode == 0 && fi) ? wv * ri : 0.0;
            const double wj = (mode == 0 && fj) ? wv * rj : 0.0;
            const double dw = wi - wj;
            const double s2 = r2 + dw * dw;
            if (s2 >= a.G.rc_max2) continue;
            const double g = (mode == 0 && fi != fj) ? gs : 1.0;
            pair_u_f64(a.G, cc, s2, g, ulj, uc, fs);
            ulj_s += 0.5 * ulj;
            uc_s += 0.5 * uc;
            vir_s += 0.5 * fs * r2;
        }
        if (s == 0 && !fi) {
            const double4 v = a.vel[b][w];
            k_s = 0.5 * a.mass[ti] * (v.x * v.x + v.y * v.y + v.z * v.z) / a.G.accel;
        }
    }
    const int wave = threadIdx.x / kWave;
    ulj_s = wave_sum(ulj_s); uc_s = wave_sum(uc_s); k_s = wave_sum(k_s); vir_s = wave_sum(vir_s);
    fly_s = wave_sum(fly_s);
    if (lane == 0) {
        red[0][wave] = ulj_s; red[1][wave] = uc_s; red[2][wave] = k_s; red[3][wave] = vir_s;
        red[4][wave] = fly_s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double sum = 0.0;
        for (int q = 0; q < kBlock / kWave; ++q) sum += red[threadIdx.x][q];
        a.partial[(size_t)blockIdx.x * 5 + threadIdx.x] = sum;
    }
}

// one block per box: sum the box's k_energy blocks in a fixed order
__global__ __launch_bounds__(kBlock) void k_energy_final(KArgs a, int which) {
    __shared__ double red[5][kBlock];
    const Box &B = a.box[blockIdx.x];
    Ctl *c = a.ctl + blockIdx.x;
    const int P = kBlock >> a.lanes_log2;
    const int lo = B.a0 / P, hi = (B.a0 + B.cap) / P;
    for (int comp = 0; comp < 5; ++comp) {
        double s = 0.0;
        for (int q = lo + threadIdx.x; q < hi; q += kBlock) s += a.partial[(size_t)q * 5 + comp];
        red[comp][threadIdx.x] = s;
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int comp = 0; comp < 5; ++comp) red[comp][threadIdx.x] += red[comp][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double U = red[0][0] + red[1][0];
        if (which == 0) { c->U0 = U; c->K0 = red[2][0]; c->Ufly0 = red[4][0]; }
        else if (which == 1) { c->U1 = U; c->K1 = red[2][0]; c->Ufly1 = red[4][0]; }
        c->Ulj = red[0][0]; c->Uc = red[1][0]; c->vir = red[3][0];
    }
}

// ==========================================================================
// Metropolis test, Eqs. (6) and (8), one thread per box:
// ln R = -beta dH +- (beta mu + I), I = 2 ln(V / (Lambda_s^3 (N + 1))),
// N the pair count of the smaller state.
// ==========================================================================
__global__ void k_metropolis(KArgs a) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= a.nbox) return;
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    TrialRec *r = a.rec + bi;
    const int move = c->move;
    r->trial = c->trial;
    r->n_atoms = c->n;
    r->n_salt_before = c->nsalt;
    r->n_salt_after = c->nsalt;
    r->n_steps = c->nf;
    r->ln_u = log(c->u[7]);
    r->ln_proposal = c->lnq;
    r->flags = 0;
    r->accepted = 0;
    c->accepted = 0;
    if ((c->err & (kErrNbr | kErrCell | kErrSkin | kErrCap | kErrFast)) && !(c->err & kErrNonfinite)) c->retry = 1;
    if (move == 0) {
        r->move = -1;
        r->flags = c->idle ? kFlagIdle : (c->retry ? 0u : kFlagEmpty);
        r->tag_c = r->tag_a = -1;
        r->dH = r->dU = r->dK = r->W_prot = r->E_switch = r->dM = 0.0;
        r->ln_ratio = -INFINITY;
        r->H0 = r->H1 = 0.0;
        return;
    }
    if (move == kMoveMD) {
        // equilibrium phase (generalized hybrid MC): ln R = -beta dH
        const double H0 = c->U0 + c->K0, H1 = c->U1 + c->K1, dH = H1 - H0;
        r->trial = c->md;
        r->move = kMoveMD;
        r->tag_c = r->tag_a = -1;
        r->dH = dH; r->dU = c->U1 - c->U0; r->dK = c->K1 - c->K0;
        r->H0 = H0; r->H1 = H1;
        r->W_prot = r->E_switch = r->dM = 0.0;
        r->ln_ratio = -a.G.beta * dH;
        int acc = 0;
        if (!isfinite(dH) || (c->err & kErrNonfinite)) r->flags |= kFlagNonfinite;
        else acc = r->ln_u < r->ln_ratio;
        if (c->retry) acc = 0;
        r->accepted = acc;
        c->accepted = acc;
        return;
    }
    r->move = move;
    if (c->instant) r->flags |= kFlagInstant;
    r->tag_c = a.ctag[c->ic];
    r->tag_a = a.ctag[c->ia];
    const double H0 = c->U0 + c->K0, H1 = c->U1 + c->K1;
    const double dH = H1 - H0;
    const int n_small = move > 0 ? c->nsalt : c->nsalt - 1;
    const double I = 2.0 * log(B.volume / (a.G.lambda3 * (double)(n_small + 1)));
    const double lnR = (move > 0 ? -a.G.beta * dH + a.G.beta_mu + I : -a.G.beta * dH - a.G.beta_mu - I) + c->lnq;
    r->dH = dH; r->dU = c->U1 - c->U0; r->dK = c->K1 - c->K0;
    r->H0 = H0; r->H1 = H1;
    r->W_prot = c->Wf[0] + c->Wf[1];
    r->E_switch = move > 0 ? c->Ufly0 : -c->Ufly1;
    r->dM = move > 0 ? dH - I / a.G.beta : -dH - I / a.G.beta;
    r->ln_ratio = lnR;
    int acc = 0;
    if (!isfinite(dH) || (c->err & kErrNonfinite)) r->flags |= kFlagNonfinite;
    else acc = r->ln_u < lnR;
    if (c->retry) acc = 0;
    r->accepted = acc;
    c->accepted = acc;
}

// Bimodal bias, insertion (Eq. 15): ln of B_del / B_ins = (N + 1) / W, W the
// sum of B_ins(r_a, r_c) over the anions of the (N+1)-state the trajectory
// reached (final working buffer, the cation fixed in 3D); one block per box,
// chunk sums combined in a fixed order.
__global__ __launch_bounds__(kBlock) void k_bias_end(KArgs a) {
    const int bi = blockIdx.x, tid = threadIdx.x;
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    if (c->move != 1 || a.G.bias_alpha <= 0.0) return;
    __shared__ double s_w[kBlock];
    const int b = buf_of(-1, c);
    const double4 pc = a.pos[b][c->wic];
    const int n = c->n_all;
    const int chunk = (n + kBlock - 1) / kBlock;
    const int lo = B.a0 + tid * chunk, hi = B.a0 + min(n, tid * chunk + chunk);
    double part = 0.0;
    for (int i = lo; i < hi; ++i) {
        const double4 p = a.pos[b][i];
        if ((meta_of(p) & kTypeMask) == a.anion_type) part += bias_B(a, B, p, pc);
    }
    s_w[tid] = part;
    __syncthreads();
    if (tid == 0) {
        double W = 0.0;
        for (int q = 0; q < kBlock; ++q) W += s_w[q];
        c->lnq = log((double)(c->nsalt + 1)) - log(W);
    }
}

// Commit (accepted: the working positions go back to canonical order, ghosts
// become physical, a deleted pair is compacted out) or roll back (the
// canonical arrays are the snapshot; only a deletion's flags are cleared).
// Carried momenta: an accepted trial's end momenta (times the end reversal
// sign) become the state's, a rejected trial's keep both reversal signs; an
// equilibrium phase keeps its end momenta, or reverses its refreshed ones.
__global__ __launch_bounds__(kBlock) void k_commit(KArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    const int move = c->move;
    if (move == 0) return;
    const bool carry = a.G.momenta != 0 || move == kMoveMD;
    if (c->accepted) {
        if (i - B.a0 < c->n_all) {
            const int e = buf_of(-1, c);
            const double4 p = a.pos[e][i];
            a.cpos[a.perm[i]] = with_meta(p.x, p.y, p.z, meta_of(p) & kTypeMask);
            if (carry) {
                const double s1 = move == kMoveMD ? 1.0 : reversal_sign(a, B, c->trial, 1);
                const double4 v = a.vel[e][i];
                a.cvel[a.perm[i]] = make_double4(s1 * v.x, s1 * v.y, s1 * v.z, 0.0);
            }
        }
        return;
    }
    if (carry && !c->retry && i - B.a0 < c->n) {   // (a trial to recompute keeps its start state)
        if (move == kMoveMD) {
            const double4 v = refreshed_velocity(a, B, c, i);
            a.cvel[i] = make_double4(-v.x, -v.y, -v.z, 0.0);
        } else {
            const double s = reversal_sign(a, B, c->trial, 0) * reversal_sign(a, B, c->trial, 1);
            const double4 v = a.cvel[i];
            a.cvel[i] = make_double4(s * v.x, s * v.y, s * v.z, 0.0);
        }
    }
    if (move < 0 && i == B.a0) {
        double4 p = a.cpos[c->ic];
        a.cpos[c->ic] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
        p = a.cpos[c->ia];
        a.cpos[c->ia] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
    }
}

// accepted deletion: stable compaction of the canonical arrays without the pair
__global__ __launch_bounds__(kBlock) void k_compact1(KArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    if (!(c->accepted && c->move < 0)) return;
    const int ic = c->ic, ia = c->ia;
    if (i - B.a0 < c->n_all && i != ic && i != ia) {
        const int d = i - (i > ic) - (i > ia);
        a.tpos[d] = a.cpos[i];
        a.tvel[d] = a.cvel[i];
        a.ttag[d] = a.ctag[i];
        a.ttype[d] = a.ctype[i];
        a.tmol[d] = a.cmol[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_compact2(KArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    if (!(c->accepted && c->move < 0)) return;
    if (i - B.a0 < c->n_all - 2) {
        a.cpos[i] = a.tpos[i];
        a.cvel[i] = a.tvel[i];
        a.ctag[i] = a.ttag[i];
        a.ctype[i] = a.ttype[i];
        a.cmol[i] = a.tmol[i];
    }
}

__global__ void k_commit_ctl(KArgs a) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= a.nbox) return;
    Ctl *c = a.ctl + bi;
    TrialRec *r = a.rec + bi;
    if (c->accepted) {
        if (c->move == 1) { c->n += 2; c->nsalt += 1; c->next_tag += 2; }
        else if (c->move == -1) { c->n -= 2; c->nsalt -= 1; }
    }
    c->n_all = c->n;
    r->n_salt_after = c->nsalt;
    if (c->move == kMoveMD) { if (!c->retry) c->md += 1; }
    else if (!c->retry && !c->idle) c->trial += 1;
}

// Every box runs `count` more equilibrium phases in a phase round and then
// idles.
__global__ void k_set_md_quota(KArgs a, long long count) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= a.nbox) return;
    Ctl *c = a.ctl + bi;
    c->md_end = c->md + count;
}

// Momenta of the state at set-up: a Maxwell-Boltzmann draw for every atom
// (counter 0 of its own stream).
__global__ __launch_bounds__(kBlock) void k_init_velocities(KArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.slots) return;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    if (i - B.a0 >= a.ctl[bi].n) return;
    a.cvel[i] = mb_velocity(a, B, 0, kPurposeInitV, a.ctag[i], sqrt(a.G.accel * a.G.kT / a.mass[a.ctype[i]]));
}

// Every box runs `count` more trials and then idles (count < 0: no limit).
__global__ void k_set_quota(KArgs a, long long count) {
    const int bi = blockIdx.x * blockDim.x + threadIdx.x;
    if (bi >= a.nbox) return;
    Ctl *c = a.ctl + bi;
    c->trial_end = count < 0 ? 0x7fffffffffffffffLL : c->trial + count;
}

// Speculative trials: every box of the batch takes box src's state between
// trials (canonical arrays, atom and pair counts, next tag).  The boxes are
// replicas of one chain with equal capacities.
__global__ __launch_bounds__(kBlock) void k_broadcast_box(KArgs a, int src) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.slots) return;
    const int bi = box_of_slot(a, i);
    if (bi == src) return;
    const Ctl *cs = a.ctl + src;
    const int o = i - a.box[bi].a0;
    if (o < cs->n) {
        const int j = a.box[src].a0 + o;
        a.cpos[i] = a.cpos[j];
        a.cvel[i] = a.cvel[j];
        a.ctag[i] = a.ctag[j];
        a.ctype[i] = a.ctype[j];
        a.cmol[i] = a.cmol[j];
    }
    if (o == 0) {
        Ctl *c = a.ctl + bi;
        c->n = cs->n;
        c->n_all = cs->n_all;
        c->nsalt = cs->nsalt;
        c->next_tag = cs->next_tag;
        c->md = cs->md;
    }
}

// Sum of list lengths of the current states (for the roofline byte count).
__global__ __launch_bounds__(kBlock) void k_sum_nbr(KArgs a, unsigned long long *out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    unsigned long long v = (i - B.a0 < a.ctl[bi].n_all) ? (unsigned long long)a.nnbr[i] : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x % kWave) == 0) atomicAdd(out, v);
}

// Test hooks on the canonical state: flag an atom slot as flying or not.
__global__ void k_set_fly(KArgs a, int i, int on) {
    double4 p = a.cpos[i];
    int m = meta_of(p);
    m = on ? (m | kFlyBit) : (m & ~kFlyBit);
    a.cpos[i] = with_meta(p.x, p.y, p.z, m);
}

// ==========================================================================
// Rigid water.  Velocity constraint (RATTLE): remove from the three atoms'
// velocities the components that would change a bond length, by solving the
// 3x3 system for the multipliers of the bonds O-H1, O-H2, H1-H2 (Cramer).
// Positions (SETTLE): the constrained triangle is the rigid canonical one
// with the centre of mass of the unconstrained positions, the same
// components normal to the old plane (the corrections act along old bonds),
// and no torque of the corrections about the old positions; those fix the
// two tilts and the in-plane angle in closed form.
// ==========================================================================
struct d3 { double x, y, z; };
__device__ __forceinline__ d3 mk(double x, double y, double z) { d3 r; r.x = x; r.y = y; r.z = z; return r; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ d3 unit(d3 a) { return (1.0 / sqrt(dot(a, a))) * a; }

__device__ __forceinline__ void rattle_velocities(const Geo &G, const d3 &a, const d3 &b, const d3 &c,
                                                  d3 &va, d3 &vb, d3 &vc) {
    const double io = 1.0 / G.m_o, ih = 1.0 / G.m_h;
    const d3 rab = a - b, rac = a - c, rbc = b - c;
    const double M11 = (io + ih) * dot(rab, rab), M12 = io * dot(rac, rab), M13 = -ih * dot(rbc, rab);
    const double M21 = io * dot(rab, rac), M22 = (io + ih) * dot(rac, rac), M23 = ih * dot(rbc, rac);
    const double M31 = -ih * dot(rab, rbc), M32 = ih * dot(rac, rbc), M33 = 2.0 * ih * dot(rbc, rbc);
    const double r1 = -dot(va - vb, rab), r2 = -dot(va - vc, rac), r3 = -dot(vb - vc, rbc);
    const double det = M11 * (M22 * M33 - M23 * M32) - M12 * (M21 * M33 - M23 * M31) + M13 * (M21 * M32 - M22 * M31);
    const double l1 = (r1 * (M22 * M33 - M23 * M32) - M12 * (r2 * M33 - M23 * r3) + M13 * (r2 * M32 - M22 * r3)) / det;
    const double l2 = (M11 * (r2 * M33 - M23 * r3) - r1 * (M21 * M33 - M23 * M31) + M13 * (M21 * r3 - r2 * M31)) / det;
    const double l3 = (M11 * (M22 * r3 - r2 * M32) - M12 * (M21 * r3 - r2 * M31) + r1 * (M21 * M32 - M22 * M31)) / det;
    va = va + io * (l1 * rab + l2 * rac);
    vb = vb + ih * (l3 * rbc - l1 * rab);
    vc = vc - ih * (l2 * rac + l3 * rbc);
}

// old: a0, b0, c0 (constrained); in/out: a1, b1, c1 (unconstrained -> constrained)
__device__ __forceinline__ void settle_positions(const Geo &G, const d3 &a0, const d3 &b0, const d3 &c0,
                                                 d3 &a1, d3 &b1, d3 &c1) {
    const double mo = G.m_o, mh = G.m_h, Mt = mo + 2.0 * mh;
    // frame of the old molecule: x from H1 to H2, y towards O, z normal
    const d3 ex = unit(c0 - b0);
    d3 ey = a0 - 0.5 * (b0 + c0);
    ey = unit(ey - dot(ey, ex) * ex);
    const d3 ez = cross(ex, ey);
    const d3 d0 = (1.0 / Mt) * (mo * a0 + mh * (b0 + c0));
    const d3 d1 = (1.0 / Mt) * (mo * a1 + mh * (b1 + c1));
    const d3 A0 = a0 - d0, B0 = b0 - d0, C0 = c0 - d0;
    const d3 A1 = a1 - d1, B1 = b1 - d1, C1 = c1 - d1;
    const double X0[3] = {dot(A0, ex), dot(B0, ex), dot(C0, ex)};
    const double Y0[3] = {dot(A0, ey), dot(B0, ey), dot(C0, ey)};
    const double X1[3] = {dot(A1, ex), dot(B1, ex), dot(C1, ex)};
    const double Y1[3] = {dot(A1, ey), dot(B1, ey), dot(C1, ey)};
    const double zA = dot(A1, ez), zB = dot(B1, ez), zC = dot(C1, ez);
    const double ra = G.ra, rb = G.rb, rc = G.rc_w;
    const double sphi = zA / ra, cphi = sqrt(fmax(0.0, 1.0 - sphi * sphi));
    const double spsi = (zB - zC) / (2.0 * rc * cphi), cpsi = sqrt(fmax(0.0, 1.0 - spsi * spsi));
    // canonical triangle tilted about y (psi) then x (phi)
    const double Qx[3] = {0.0, -rc * cpsi, rc * cpsi};
    const double Qy[3] = {ra * cphi, -rb * cphi - rc * spsi * sphi, -rb * cphi + rc * spsi * sphi};
    const double Qz[3] = {ra * sphi, -rb * sphi + rc * spsi * cphi, -rb * sphi - rc * spsi * cphi};
    const double m[3] = {mo, mh, mh};
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = 0; i < 3; ++i) {
        al += m[i] * (X0[i] * Qx[i] + Y0[i] * Qy[i]);
        be += m[i] * (X0[i] * Qy[i] - Y0[i] * Qx[i]);
        ga += m[i] * (X0[i] * Y1[i] - Y0[i] * X1[i]);
    }
    const double n2 = al * al + be * be;
    const double sd = sqrt(fmax(0.0, n2 - ga * ga));
    const double sth = (al * ga - be * sd) / n2, cth = (be * ga + al * sd) / n2;
    d3 out[3];
    for (int i = 0; i < 3; ++i) {
        const double px = Qx[i] * cth - Qy[i] * sth, py = Qx[i] * sth + Qy[i] * cth;
        out[i] = d1 + px * ex + py * ey + Qz[i] * ez;
    }
    a1 = out[0]; b1 = out[1]; c1 = out[2];
}

__device__ __forceinline__ d3 unwrap_near(const Box &B, const double4 &p, const d3 &ref) {
    return mk(ref.x + min_image(p.x - ref.x, B.L[0]), ref.y + min_image(p.y - ref.y, B.L[1]),
              ref.z + min_image(p.z - ref.z, B.L[2]));
}

// Rigid waters: every box holds n_mol of them as its first atoms (canonical
// slots a0 + 3m + q, q = O, H, H); one thread per molecule of every box.
__device__ __forceinline__ int water_slots(const KArgs &a, int gm, int w[3]) {
    const int bi = gm / a.G.n_mol, m = gm - bi * a.G.n_mol;
    const int c0 = a.box[bi].a0 + 3 * m;
    w[0] = a.molw[c0]; w[1] = a.molw[c0 + 1]; w[2] = a.molw[c0 + 2];
    return bi;
}

// trial start: project the freshly drawn water velocities (working buffer 0)
__global__ __launch_bounds__(kBlock) void k_rattle_mb(KArgs a) {
    const int gm = blockIdx.x * kBlock + threadIdx.x;
    if (gm >= a.G.n_mol * a.nbox) return;
    int w[3];
    const Box &B = a.box[water_slots(a, gm, w)];
    const double4 pa = a.pos[0][w[0]];
    const d3 ra_ = mk(pa.x, pa.y, pa.z);
    const d3 x1 = unwrap_near(B, a.pos[0][w[1]], ra_), x2 = unwrap_near(B, a.pos[0][w[2]], ra_);
    double4 v4[3] = {a.vel[0][w[0]], a.vel[0][w[1]], a.vel[0][w[2]]};
    d3 v[3];
    for (int i = 0; i < 3; ++i) v[i] = mk(v4[i].x, v4[i].y, v4[i].z);
    rattle_velocities(a.G, ra_, x1, x2, v[0], v[1], v[2]);
    for (int i = 0; i < 3; ++i) a.vel[0][w[i]] = make_double4(v[i].x, v[i].y, v[i].z, 0.0);
}

// Rigid waters' canonical momenta restricted to the constraint surface (the
// velocity constraint on the canonical positions), one thread per molecule
// of every box: at set-up, and (rejected_phase_only) after a rejected
// equilibrium phase, whose reversed refresh k_commit wrote unrestricted --
// the restriction is linear, so this gives the reversed momenta the phase's
// trajectory started from.
__global__ __launch_bounds__(kBlock) void k_water_cvel(KArgs a, int rejected_phase_only) {
    const int gm = blockIdx.x * kBlock + threadIdx.x;
    if (gm >= a.G.n_mol * a.nbox) return;
    const int bi = gm / a.G.n_mol, m = gm - bi * a.G.n_mol;
    const Box &B = a.box[bi];
    const Ctl *c = a.ctl + bi;
    if (rejected_phase_only && !(c->move == kMoveMD && !c->accepted && !c->retry)) return;
    const int i0 = B.a0 + 3 * m;
    const double4 pa = a.cpos[i0];
    const d3 ra_ = mk(pa.x, pa.y, pa.z);
    const d3 x1 = unwrap_near(B, a.cpos[i0 + 1], ra_), x2 = unwrap_near(B, a.cpos[i0 + 2], ra_);
    d3 v[3];
    for (int q = 0; q < 3; ++q) {
        const double4 v4 = a.cvel[i0 + q];
        v[q] = mk(v4.x, v4.y, v4.z);
    }
    rattle_velocities(a.G, ra_, x1, x2, v[0], v[1], v[2]);
    for (int q = 0; q < 3; ++q) a.cvel[i0 + q] = make_double4(v[q].x, v[q].y, v[q].z, 0.0);
}

// One step k of the rigid waters (after k_step stored their forces F_k):
// v_k = v + h F/m and the velocity constraint (k > 0); v += h F/m, drift and
// position constraint with its velocity correction (k < nf).
// (one thread per molecule in blocks of one wavefront, so that the few
// thousand molecules of a box spread over many CUs)
constexpr int kSettleBlock = 64;

__global__ __launch_bounds__(kSettleBlock) void k_settle(KArgs a, int k, int b0, int bin, int cl) {
    const int gm = blockIdx.x * kSettleBlock + threadIdx.x;
    if (gm >= a.G.n_mol * a.nbox) return;
    int w[3];
    const int bi = water_slots(a, gm, w);
    const Box &B = a.box[bi];
    Ctl *c = a.ctl + bi;
    const int move = c->move, nf = c->nf;
    if (move == 0 || k > nf) return;
    const int b = buf_of(b0, c);
    int *fast = a.fast + (size_t)bi * 3 * kFastCap;
    const Geo &G = a.G;
    double4 p4[3], v4[3], f4[3];
    for (int i = 0; i < 3; ++i) { p4[i] = a.pos[b][w[i]]; v4[i] = a.vel[b][w[i]]; f4[i] = a.fw[w[i]]; }
    const d3 x0[3] = {mk(p4[0].x, p4[0].y, p4[0].z), unwrap_near(B, p4[1], mk(p4[0].x, p4[0].y, p4[0].z)),
                      unwrap_near(B, p4[2], mk(p4[0].x, p4[0].y, p4[0].z))};
    d3 v[3];
    double hm[3];
    for (int i = 0; i < 3; ++i) {
        v[i] = mk(v4[i].x, v4[i].y, v4[i].z);
        hm[i] = G.half_dt * G.accel / a.mass[meta_of(p4[i]) & kTypeMask];
    }
    if (k > 0) {
        for (int i = 0; i < 3; ++i) v[i] = v[i] + hm[i] * mk(f4[i].x, f4[i].y, f4[i].z);
        rattle_velocities(G, x0[0], x0[1], x0[2], v[0], v[1], v[2]);
    }
    d3 x[3] = {x0[0], x0[1], x0[2]};
    if (k < nf) {
        d3 xu[3];
        for (int i = 0; i < 3; ++i) {
            v[i] = v[i] + hm[i] * mk(f4[i].x, f4[i].y, f4[i].z);
            xu[i] = x0[i] + G.dt * v[i];
            x[i] = xu[i];
        }
        settle_positions(G, x0[0], x0[1], x0[2], x[0], x[1], x[2]);
        for (int i = 0; i < 3; ++i) v[i] = v[i] + (1.0 / G.dt) * (x[i] - xu[i]);
    }
    const int lw = (k + 1) % 3;
    for (int i = 0; i < 3; ++i) {
        const double px = wrap_coord(x[i].x, B.L[0]), py = wrap_coord(x[i].y, B.L[1]), pz = wrap_coord(x[i].z, B.L[2]);
        int mo = meta_of(p4[i]);
        uint4 qn = fixed_of(B, px, py, pz, mo);
        if ((mo & kFastBit) == 0 && moved_beyond_half_skin(a, B, qn, a.posb[w[i]])) mo |= kFastBit;
        if (mo & kFastBit) {
            const int slot = atomicAdd(&c->nfast[lw], 1);
            if (slot < kFastCap) fast[lw * kFastCap + slot] = w[i];
            else atomicOr(&c->err, kErrFast);
            atomicMax(&c->max_fast, slot + 1);
        }
        qn.w = (unsigned)mo;
        const double4 pn = with_meta(px, py, pz, mo);
        a.pos[b ^ 1][w[i]] = pn;
        a.fx[b ^ 1][w[i]] = qn;
        a.vel[b ^ 1][w[i]] = make_double4(v[i].x, v[i].y, v[i].z, 0.0);
        if (bin && k < nf) bin_atom(a, B, c, cl ^ 1, w[i], pn);
    }
}

}  // namespace h4d
