// h4d_kernels.hpp -- HIP kernels of one H4D exchange trial on gfx950.
//
// Layout in HBM (capacity cap atoms, structure of arrays):
//   pos[2]   double4 ping-pong buffers: x, y, z (FP64, wrapped) + meta word
//   fx[2]    uint4 ping-pong buffers: 32-bit fixed-point x, y, z + meta word
//            (FP32 mode: the pair pass gathers these 16-byte records)
//   vel      double4
//   tag/type/mol  per atom; array order = ascending tag order
//   nbr      column-major ELL Verlet list nbr[q * cap + i], counts nnbr[i]
//   cells    cell_cnt[c], cell_atoms[c * cell_cap + slot] (sorted per cell)
// Every kernel reads the atom counts from the control block, so a trial's
// launches never wait on the host.
#pragma once
#include "h4d_device.hpp"

namespace h4d {

struct Ctl {
    int n;            // atoms of the physical state
    int n_all;        // atoms including the two ghosts of an insertion
    int nsalt;
    int move;         // +1 insertion, -1 deletion, 0 nothing to do
    int ic, ia;       // indices of the flying cation / anion
    int nf;           // NEMD steps of this trial
    int accepted;
    unsigned err;     // kErr* bits of this trial
    unsigned retry;   // 1: the trial must be recomputed
    int max_nbr, max_cell;
    long long next_tag;
    long long trial;
    double u[8];
    double U0, K0, U1, K1;
    double Ulj, Uc, vir;
    double Wf[2], Esw[2], Esw_pair;
};

// Trial record, same layout as h4d_trial of the C ABI.
struct TrialRec {
    int move, accepted, n_salt_before, n_salt_after, n_steps;
    unsigned flags;
    int n_atoms, n_rebuilds;
    long long trial, tag_c, tag_a;
    double dH, dU, dK, W_prot, E_switch, dM, ln_ratio, ln_u, ln_proposal, H0, H1;
};

struct KArgs {
    Geo G;
    const PairCoef *coef;
    double4 *pos[2];
    uint4 *fx[2];
    double4 *vel;
    double4 *pos0;       // snapshot of the trial's starting positions
    double4 *posb;       // positions at the last list build
    double4 *force;      // test hook output / rigid-water scratch
    long long *tag;
    int *type;
    int *mol;
    double4 *tpos;       // compaction scratch
    long long *ttag;
    int *ttype, *tmol;
    int *nbr, *nnbr;
    int *cell_cnt, *cell_atoms;
    double *partial;     // per-block FP64 partial sums, 4 per block
    Ctl *ctl;
    TrialRec *rec;
    const double *mass;  // per type
    int cap, nbr_cap, cell_cap, ncell_total;
    uint64_t seed, stream;
    int n_steps, n_steps_min, n_steps_max;
    int cation_type, anion_type;
};

// Coefficients are staged in LDS once per block.
struct CoefLds {
    PairCoef c[kMaxTypes * kMaxTypes];
};

__device__ __forceinline__ void load_coef(CoefLds &s, const PairCoef *g, int nt) {
    for (int q = threadIdx.x; q < kMaxTypes * kMaxTypes; q += blockDim.x) s.c[q] = g[q];
    (void)nt;
}

// ==========================================================================
// Proposal: move choice, ghost pair for an insertion, rank selection for a
// deletion (Eqs. 3-4; uniform 1/2 between the two moves).
// ==========================================================================
__global__ __launch_bounds__(kBlock) void k_propose(KArgs a, int force_move) {
    Ctl *c = a.ctl;
    __shared__ int s_cnt[2][kBlock];
    __shared__ int s_move, s_kc, s_ka, s_ic, s_ia, s_n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const uint64_t t = (uint64_t)c->trial;
        const u64x4 r0 = philox(t, kPurposeSelect, 0, 0, a.seed, a.stream);
        const u64x4 r1 = philox(t, kPurposeSelect, 1, 0, a.seed, a.stream);
        for (int q = 0; q < 4; ++q) { c->u[q] = unit_open(r0.v[q]); c->u[4 + q] = unit_open(r1.v[q]); }
        int nf = a.n_steps;
        if (a.n_steps_max > 0) {
            const u64x4 rn = philox(t, kPurposeNsteps, 0, 0, a.seed, a.stream);
            nf = a.n_steps_min + (int)floor(unit_open(rn.v[0]) * (double)(a.n_steps_max - a.n_steps_min + 1));
        }
        c->nf = nf;
        int move = force_move ? force_move : (c->u[0] < 0.5 ? 1 : -1);
        if (move < 0 && c->nsalt == 0) move = 0;
        c->move = move;
        c->err = 0; c->retry = 0; c->accepted = 0;
        c->Wf[0] = c->Wf[1] = 0.0; c->Esw[0] = c->Esw[1] = 0.0; c->Esw_pair = 0.0;
        c->ic = c->ia = -1;
        c->n_all = c->n;
        s_move = move; s_n = c->n;
        s_kc = (int)floor(c->u[1] * (double)c->nsalt);
        s_ka = (int)floor(c->u[2] * (double)c->nsalt);
        s_ic = s_ia = -1;
        if (move > 0) {
            const int n = c->n;
            if (n + 2 > a.cap) {
                c->err |= kErrCap; c->retry = 1; c->move = 0; s_move = 0;
            } else {
                const int ic = n, ia = n + 1;
                const int tcat = a.cation_type, tan = a.anion_type;
                const double xc[3] = {wrap_coord(a.G.L[0] * c->u[1], a.G.L[0]),
                                      wrap_coord(a.G.L[1] * c->u[2], a.G.L[1]),
                                      wrap_coord(a.G.L[2] * c->u[3], a.G.L[2])};
                const double xa[3] = {wrap_coord(a.G.L[0] * c->u[4], a.G.L[0]),
                                      wrap_coord(a.G.L[1] * c->u[5], a.G.L[1]),
                                      wrap_coord(a.G.L[2] * c->u[6], a.G.L[2])};
                a.pos[0][ic] = with_meta(xc[0], xc[1], xc[2], tcat | kFlyBit);
                a.pos[0][ia] = with_meta(xa[0], xa[1], xa[2], tan | kFlyBit);
                a.tag[ic] = c->next_tag; a.tag[ia] = c->next_tag + 1;
                a.type[ic] = tcat; a.type[ia] = tan;
                a.mol[ic] = -1; a.mol[ia] = -1;
                c->ic = ic; c->ia = ia; c->n_all = n + 2;
            }
        }
    }
    __syncthreads();
    if (s_move >= 0) return;
    // deletion: the atom of each species with the drawn rank in tag order;
    // array order is tag order, so count species members per chunk and scan
    const int n = s_n;
    const int chunk = (n + kBlock - 1) / kBlock;
    const int lo = tid * chunk, hi = min(n, lo + chunk);
    int nc = 0, na = 0;
    for (int i = lo; i < hi; ++i) {
        const int ty = a.type[i];
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
    int pc = s_cnt[0][tid], pa = s_cnt[1][tid];
    if (s_kc >= pc && s_kc < pc + nc) {
        int r = pc;
        for (int i = lo; i < hi; ++i)
            if (a.type[i] == a.cation_type) { if (r == s_kc) { s_ic = i; break; } ++r; }
    }
    if (s_ka >= pa && s_ka < pa + na) {
        int r = pa;
        for (int i = lo; i < hi; ++i)
            if (a.type[i] == a.anion_type) { if (r == s_ka) { s_ia = i; break; } ++r; }
    }
    __syncthreads();
    if (tid == 0) {
        const int ic = s_ic, ia = s_ia;
        if (ic < 0 || ia < 0) {   // species counts disagree with nsalt: refuse the move
            c->err |= kErrCap; c->retry = 1; c->move = 0;
            return;
        }
        c->ic = ic; c->ia = ia;
        double4 p = a.pos[0][ic];
        a.pos[0][ic] = with_meta(p.x, p.y, p.z, meta_of(p) | kFlyBit);
        p = a.pos[0][ia];
        a.pos[0][ia] = with_meta(p.x, p.y, p.z, meta_of(p) | kFlyBit);
    }
}

// ==========================================================================
// Maxwell-Boltzmann momenta keyed by tag (Box-Muller on Philox uniforms);
// also refreshes the fixed-point coordinates of buffer 0.
// ==========================================================================
__global__ __launch_bounds__(kBlock) void k_mb(KArgs a) {
    const Ctl *c = a.ctl;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= c->n_all) return;
    const uint64_t t = (uint64_t)c->trial;
    const u64x4 r = philox(t, kPurposeMB, (uint64_t)a.tag[i], 0, a.seed, a.stream);
    const double u0 = unit_open(r.v[0]), u1 = unit_open(r.v[1]);
    const double u2 = unit_open(r.v[2]), u3 = unit_open(r.v[3]);
    const double r01 = sqrt(-2.0 * log(u0)), r23 = sqrt(-2.0 * log(u2));
    const double twopi = 6.283185307179586476925286766559;
    const double4 p = a.pos[0][i];
    const int ty = meta_of(p) & kTypeMask;
    const double sd = sqrt(a.G.accel * a.G.kT / a.mass[ty]);
    a.vel[i] = make_double4(sd * (r01 * cos(twopi * u1)), sd * (r01 * sin(twopi * u1)),
                            sd * (r23 * cos(twopi * u3)), 0.0);
    a.fx[0][i] = make_uint4(to_fixed(p.x, a.G.fx_inv[0]), to_fixed(p.y, a.G.fx_inv[1]),
                            to_fixed(p.z, a.G.fx_inv[2]), (unsigned)meta_of(p));
}

// ==========================================================================
// Cell and Verlet lists.
// ==========================================================================
__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
    int k = (int)(x / L * (double)nc);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

__global__ void k_cell_clear(KArgs a, int k_step) {
    if (k_step > a.ctl->nf) return;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.ncell_total) a.cell_cnt[q] = 0;
}

__global__ __launch_bounds__(kBlock) void k_cell_bin(KArgs a, int b, int k_step) {
    const Ctl *c = a.ctl;
    if (k_step > c->nf) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= c->n_all) return;
    const double4 p = a.pos[b][i];
    const int cx = cell_coord(p.x, a.G.L[0], a.G.ncell[0]);
    const int cy = cell_coord(p.y, a.G.L[1], a.G.ncell[1]);
    const int cz = cell_coord(p.z, a.G.L[2], a.G.ncell[2]);
    const int cc = (cz * a.G.ncell[1] + cy) * a.G.ncell[0] + cx;
    const int slot = atomicAdd(&a.cell_cnt[cc], 1);
    if (slot < a.cell_cap) a.cell_atoms[(size_t)cc * a.cell_cap + slot] = i;
    else { atomicOr(&a.ctl->err, kErrCell); atomicMax(&a.ctl->max_cell, slot + 1); }
}

// Sort each cell's atom indices ascending (rank sort in LDS), so the list
// order does not depend on the order of the binning atomics.
__global__ __launch_bounds__(kWave) void k_cell_sort(KArgs a, int k_step) {
    if (k_step > a.ctl->nf) return;
    extern __shared__ int buf[];
    const int cc = blockIdx.x;
    const int cnt = min(a.cell_cnt[cc], a.cell_cap);
    int *row = a.cell_atoms + (size_t)cc * a.cell_cap;
    for (int q = threadIdx.x; q < cnt; q += kWave) buf[q] = row[q];
    __syncthreads();
    for (int q = threadIdx.x; q < cnt; q += kWave) {
        const int e = buf[q];
        int r = 0;
        for (int p = 0; p < cnt; ++p) r += (buf[p] < e);
        row[r] = e;
    }
}

__device__ __forceinline__ void list_try(const KArgs &a, int i, int j, int mi, const double4 &pi,
                                         const double4 *P, int &cnt) {
    if (j == i) return;
    if (mi >= 0 && a.mol[j] == mi) return;
    const double4 pj = P[j];
    const double dx = min_image(pi.x - pj.x, a.G.L[0]);
    const double dy = min_image(pi.y - pj.y, a.G.L[1]);
    const double dz = min_image(pi.z - pj.z, a.G.L[2]);
    if (dx * dx + dy * dy + dz * dz < a.G.rlist2) {
        if (cnt < a.nbr_cap) a.nbr[(size_t)cnt * a.cap + i] = j;
        ++cnt;
    }
}

__global__ __launch_bounds__(kBlock) void k_list(KArgs a, int b, int k_step) {
    const Ctl *c = a.ctl;
    if (k_step > c->nf) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int n_all = c->n_all;
    if (i >= n_all) return;
    const double4 *P = a.pos[b];
    const double4 pi = P[i];
    const int mi = a.mol[i];
    int cnt = 0;
    if (!a.G.use_cells) {
        for (int j = 0; j < n_all; ++j) list_try(a, i, j, mi, pi, P, cnt);
    } else {
        const int nx = a.G.ncell[0], ny = a.G.ncell[1], nz = a.G.ncell[2];
        const int cx = cell_coord(pi.x, a.G.L[0], nx);
        const int cy = cell_coord(pi.y, a.G.L[1], ny);
        const int cz = cell_coord(pi.z, a.G.L[2], nz);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int ax = (cx + dx + nx) % nx, ay = (cy + dy + ny) % ny, az = (cz + dz + nz) % nz;
                    const int cc = (az * ny + ay) * nx + ax;
                    const int m = min(a.cell_cnt[cc], a.cell_cap);
                    const int *row = a.cell_atoms + (size_t)cc * a.cell_cap;
                    for (int q = 0; q < m; ++q) list_try(a, i, row[q], mi, pi, P, cnt);
                }
    }
    a.nnbr[i] = min(cnt, a.nbr_cap);
    a.posb[i] = pi;
    if (cnt > a.nbr_cap) { atomicOr(&a.ctl->err, kErrNbr); atomicMax(&a.ctl->max_nbr, cnt); }
}

// ==========================================================================
// Force on one non-flying atom from its list, at altitude w (flyers at w).
// ==========================================================================
template <int PREC>
__device__ __forceinline__ void lane_force(const KArgs &a, const CoefLds &cf, int b, int i,
                                           const double4 &pi, int ti, double w, double gscr,
                                           double &fx, double &fy, double &fz) {
    const int nn = a.nnbr[i];
    const int *nl = a.nbr + i;
    const size_t stride = (size_t)a.cap;
    const PairCoef *crow = cf.c + ti * kMaxTypes;
    if (PREC == 1) {
        const uint4 *F = a.fx[b];
        const uint4 qi = F[i];
        const float sx = a.G.fx_scale[0], sy = a.G.fx_scale[1], sz = a.G.fx_scale[2];
        const float w2 = (float)(w * w), g = (float)gscr;
        float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 4
        for (int q = 0; q < nn; ++q) {
            const int j = nl[q * stride];
            const uint4 qj = F[j];
            const float dx = (float)(int)(qi.x - qj.x) * sx;
            const float dy = (float)(int)(qi.y - qj.y) * sy;
            const float dz = (float)(int)(qi.z - qj.z) * sz;
            const int mj = (int)qj.w;
            const bool fj = (mj & kFlyBit) != 0;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float s2 = fj ? r2 + w2 : r2;
            if (s2 < a.G.rc_max2f) {
                const float fs = pair_fs_f32(a.G, crow[mj & kTypeMask], s2, fj ? g : 1.0f);
                ax += fs * dx; ay += fs * dy; az += fs * dz;
            }
        }
        fx = ax; fy = ay; fz = az;
    } else {
        const double4 *P = a.pos[b];
        double ax = 0.0, ay = 0.0, az = 0.0;
        const double w2 = w * w;
#pragma unroll 2
        for (int q = 0; q < nn; ++q) {
            const int j = nl[q * stride];
            const double4 pj = P[j];
            const double dx = min_image(pi.x - pj.x, a.G.L[0]);
            const double dy = min_image(pi.y - pj.y, a.G.L[1]);
            const double dz = min_image(pi.z - pj.z, a.G.L[2]);
            const int mj = meta_of(pj);
            const bool fj = (mj & kFlyBit) != 0;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double s2 = fj ? r2 + w2 : r2;
            if (s2 < a.G.rc_max2) {
                const double fs = pair_fs_f64(a.G, crow[mj & kTypeMask], s2, fj ? gscr : 1.0);
                ax += fs * dx; ay += fs * dy; az += fs * dz;
            }
        }
        fx = ax; fy = ay; fz = az;
    }
    (void)ti;
}

__device__ __forceinline__ bool moved_beyond_half_skin(const KArgs &a, const double4 &p, const double4 &pb) {
    const double dx = min_image(p.x - pb.x, a.G.L[0]);
    const double dy = min_image(p.y - pb.y, a.G.L[1]);
    const double dz = min_image(p.z - pb.z, a.G.L[2]);
    return dx * dx + dy * dy + dz * dz > a.G.half_skin2;
}

// --------------------------------------------------------------------------
// Flying work of one flyer at x_k (one wavefront per flyer): the trapezoid
// share 1/2 [U_fly(x_k; w_{k+1}) - U_fly(x_k; w_{k-1})] (endpoints clamped),
// plus the switch energy U_fly(w_max) at the end where the pair sits at w_max.
// --------------------------------------------------------------------------
__device__ void flyer_work(const KArgs &a, const CoefLds &cf, int b, int k) {
    Ctl *c = a.ctl;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (wave > 1) return;
    const int move = c->move, nf = c->nf;
    if (move == 0 || k > nf) return;
    const int f = wave == 0 ? c->ic : c->ia;
    const int other = wave == 0 ? c->ia : c->ic;
    const double4 *P = a.pos[b];
    const double4 pf = P[f];
    const int tf = meta_of(pf) & kTypeMask;
    const double wlo = altitude(a.G.w_max, move, k > 0 ? k - 1 : 0, nf);
    const double whi = altitude(a.G.w_max, move, k < nf ? k + 1 : nf, nf);
    const double glo = exp(-a.G.kappa * wlo), ghi = exp(-a.G.kappa * whi);
    double slo = 0.0, shi = 0.0;
    const int nn = a.nnbr[f];
    for (int q = lane; q < nn; q += kWave) {
        const int j = a.nbr[(size_t)q * a.cap + f];
        if (j == other) continue;
        const double4 pj = P[j];
        const double dx = min_image(pf.x - pj.x, a.G.L[0]);
        const double dy = min_image(pf.y - pj.y, a.G.L[1]);
        const double dz = min_image(pf.z - pj.z, a.G.L[2]);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const PairCoef &cc = cf.c[tf * kMaxTypes + (meta_of(pj) & kTypeMask)];
        double ulj, uc, fs;
        const double s2lo = r2 + wlo * wlo;
        if (s2lo < a.G.rc_max2) { pair_u_f64(a.G, cc, s2lo, glo, ulj, uc, fs); slo += ulj + uc; }
        const double s2hi = r2 + whi * whi;
        if (s2hi < a.G.rc_max2) { pair_u_f64(a.G, cc, s2hi, ghi, ulj, uc, fs); shi += ulj + uc; }
    }
    slo = wave_sum(slo);
    shi = wave_sum(shi);
    if (lane == 0) {
        c->Wf[wave] += 0.5 * (shi - slo);
        if (k == 0 && move > 0) c->Esw[wave] = slo;        // U_fly(x_0; w_max)
        if (k == nf && move < 0) c->Esw[wave] = -shi;      // -U_fly(x_end; w_max)
        if (wave == 0 && ((k == 0 && move > 0) || (k == nf && move < 0))) {
            // the flyer-flyer pair: same altitude, 3D distance, unscreened
            const double4 po = P[other];
            const double dx = min_image(pf.x - po.x, a.G.L[0]);
            const double dy = min_image(pf.y - po.y, a.G.L[1]);
            const double dz = min_image(pf.z - po.z, a.G.L[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            double ulj = 0.0, uc = 0.0, fs;
            if (r2 < a.G.rc_max2)
                pair_u_f64(a.G, cf.c[tf * kMaxTypes + (meta_of(po) & kTypeMask)], r2, 1.0, ulj, uc, fs);
            c->Esw_pair = (move > 0 ? 1.0 : -1.0) * (ulj + uc);
        }
    }
}

// ==========================================================================
// One NEMD step k (k = 0..nf), fused: F(x_k; w_k) from the list; the second
// half kick of step k-1 (k > 0); the first half kick and drift of step k
// (k < nf) into the other buffer.  Flyers stay fixed in 3D.  The last block
// evaluates the flying work.
// ==========================================================================
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_step(KArgs a, int k, int b) {
    __shared__ CoefLds cf;
    load_coef(cf, a.coef, a.G.n_types);
    __syncthreads();
    if (blockIdx.x == gridDim.x - 1) { flyer_work(a, cf, b, k); return; }
    const Ctl *c = a.ctl;
    const int move = c->move, nf = c->nf, n_all = c->n_all;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (move == 0 || k > nf || i >= n_all) return;
    const double4 pi = a.pos[b][i];
    const int mi = meta_of(pi);
    if (mi & kFlyBit) {
        if (k < nf) {
            a.pos[b ^ 1][i] = pi;
            if (PREC == 1) a.fx[b ^ 1][i] = a.fx[b][i];
        }
        return;
    }
    if (moved_beyond_half_skin(a, pi, a.posb[i])) atomicOr(&a.ctl->err, kErrSkin);
    const int ti = mi & kTypeMask;
    const double w = altitude(a.G.w_max, move, k, nf);
    const double gscr = exp(-a.G.kappa * w);
    double fx, fy, fz;
    lane_force<PREC>(a, cf, b, i, pi, ti, w, gscr, fx, fy, fz);
    double4 v = a.vel[i];
    const double hm = a.G.half_dt * a.G.accel / a.mass[ti];
    if (k > 0) { v.x += hm * fx; v.y += hm * fy; v.z += hm * fz; }
    if (k < nf) {
        v.x += hm * fx; v.y += hm * fy; v.z += hm * fz;
        const double x = wrap_coord(pi.x + a.G.dt * v.x, a.G.L[0]);
        const double y = wrap_coord(pi.y + a.G.dt * v.y, a.G.L[1]);
        const double z = wrap_coord(pi.z + a.G.dt * v.z, a.G.L[2]);
        a.pos[b ^ 1][i] = with_meta(x, y, z, mi);
        if (PREC == 1)
            a.fx[b ^ 1][i] = make_uint4(to_fixed(x, a.G.fx_inv[0]), to_fixed(y, a.G.fx_inv[1]),
                                        to_fixed(z, a.G.fx_inv[2]), (unsigned)mi);
    }
    a.vel[i] = v;
}

// Test hook: forces of the current buffer-0 state with the flags it carries.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_forces(KArgs a, double w) {
    __shared__ CoefLds cf;
    load_coef(cf, a.coef, a.G.n_types);
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.ctl->n_all) return;
    const double4 pi = a.pos[0][i];
    const int mi = meta_of(pi);
    if (mi & kFlyBit) { a.force[i] = make_double4(0, 0, 0, 0); return; }
    double fx, fy, fz;
    lane_force<PREC>(a, cf, 0, i, pi, mi & kTypeMask, w, exp(-a.G.kappa * w), fx, fy, fz);
    a.force[i] = make_double4(fx, fy, fz, 0.0);
}

// ==========================================================================
// FP64 energies.  mode 0: flyers at altitude w (NEMD); mode 1: every pair
// with a flyer left out.  mode -1: chosen from the move (start: insertion
// excludes its ghosts; end: deletion excludes the removed pair; else all
// atoms at w = 0).  Each pair is counted half from each side.
// which: 0 start of trial, 1 end, 2 observables / test hook.
// ==========================================================================
__global__ __launch_bounds__(kBlock) void k_energy(KArgs a, int which, int mode, double w, int b) {
    __shared__ CoefLds cf;
    __shared__ double red[4][kBlock / kWave];
    load_coef(cf, a.coef, a.G.n_types);
    __syncthreads();
    const Ctl *c = a.ctl;
    const int move = c->move;
    if (mode < 0) mode = ((which == 0 && move > 0) || (which == 1 && move < 0)) ? 1 : 0;
    if (b < 0) b = (which == 1 && move != 0) ? (c->nf & 1) : 0;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double ulj_s = 0.0, uc_s = 0.0, k_s = 0.0, vir_s = 0.0;
    if (i < c->n_all) {
        const double4 *P = a.pos[b];
        const double4 pi = P[i];
        const int mi = meta_of(pi);
        const bool fi = (mi & kFlyBit) != 0;
        if (which == 1 && move != 0 && !fi && moved_beyond_half_skin(a, pi, a.posb[i]))
            atomicOr(&a.ctl->err, kErrSkin);
        const int ti = mi & kTypeMask;
        if (!(mode == 1 && fi)) {
            const double wi = (mode == 0 && fi) ? w : 0.0;
            const double gs = exp(-a.G.kappa * w);
            const int nn = a.nnbr[i];
            for (int q = 0; q < nn; ++q) {
                const int j = a.nbr[(size_t)q * a.cap + i];
                const double4 pj = P[j];
                const int mj = meta_of(pj);
                const bool fj = (mj & kFlyBit) != 0;
                if (mode == 1 && fj) continue;
                const double wj = (mode == 0 && fj) ? w : 0.0;
                const double dx = min_image(pi.x - pj.x, a.G.L[0]);
                const double dy = min_image(pi.y - pj.y, a.G.L[1]);
                const double dz = min_image(pi.z - pj.z, a.G.L[2]);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double dw = wi - wj;
                const double s2 = r2 + dw * dw;
                if (s2 >= a.G.rc_max2) continue;
                const double g = (mode == 0 && fi != fj) ? gs : 1.0;
                double ulj, uc, fs;
                pair_u_f64(a.G, cf.c[ti * kMaxTypes + (mj & kTypeMask)], s2, g, ulj, uc, fs);
                ulj_s += 0.5 * ulj;
                uc_s += 0.5 * uc;
                vir_s += 0.5 * fs * r2;
            }
        }
        if (!fi) {
            const double4 v = a.vel[i];
            k_s = 0.5 * a.mass[ti] * (v.x * v.x + v.y * v.y + v.z * v.z) / a.G.accel;
        }
    }
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    ulj_s = wave_sum(ulj_s); uc_s = wave_sum(uc_s); k_s = wave_sum(k_s); vir_s = wave_sum(vir_s);
    if (lane == 0) { red[0][wave] = ulj_s; red[1][wave] = uc_s; red[2][wave] = k_s; red[3][wave] = vir_s; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int q = 0; q < kBlock / kWave; ++q) s += red[threadIdx.x][q];
        a.partial[(size_t)blockIdx.x * 4 + threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_final(KArgs a, int which, int nblocks) {
    __shared__ double red[4][kBlock];
    for (int comp = 0; comp < 4; ++comp) {
        double s = 0.0;
        for (int q = threadIdx.x; q < nblocks; q += kBlock) s += a.partial[(size_t)q * 4 + comp];
        red[comp][threadIdx.x] = s;
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int comp = 0; comp < 4; ++comp) red[comp][threadIdx.x] += red[comp][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Ctl *c = a.ctl;
        const double U = red[0][0] + red[1][0];
        if (which == 0) { c->U0 = U; c->K0 = red[2][0]; }
        else if (which == 1) { c->U1 = U; c->K1 = red[2][0]; }
        c->Ulj = red[0][0]; c->Uc = red[1][0]; c->vir = red[3][0];
    }
}

__global__ __launch_bounds__(kBlock) void k_snapshot(KArgs a) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < a.ctl->n_all) a.pos0[i] = a.pos[0][i];
}

// ==========================================================================
// Metropolis test, Eqs. (6) and (8): ln R = -beta dH +- (beta mu + I),
// I = 2 ln(V / (Lambda_s^3 (N + 1))), N the pair count of the smaller state.
// ==========================================================================
__global__ void k_metropolis(KArgs a) {
    Ctl *c = a.ctl;
    TrialRec *r = a.rec;
    const int move = c->move;
    r->trial = c->trial;
    r->n_atoms = c->n;
    r->n_salt_before = c->nsalt;
    r->n_salt_after = c->nsalt;
    r->n_steps = c->nf;
    r->ln_u = log(c->u[7]);
    r->ln_proposal = 0.0;
    r->flags = 0;
    r->accepted = 0;
    c->accepted = 0;
    if (c->err & (kErrNbr | kErrCell | kErrSkin | kErrCap)) c->retry = 1;
    if (move == 0) {
        r->move = -1;
        r->flags = c->retry ? 0u : 1u;   // H4D_FLAG_EMPTY
        r->tag_c = r->tag_a = -1;
        r->dH = r->dU = r->dK = r->W_prot = r->E_switch = r->dM = 0.0;
        r->ln_ratio = -INFINITY;
        r->H0 = r->H1 = 0.0;
        return;
    }
    r->move = move;
    r->tag_c = a.tag[c->ic];
    r->tag_a = a.tag[c->ia];
    const double H0 = c->U0 + c->K0, H1 = c->U1 + c->K1;
    const double dH = H1 - H0;
    const int n_small = move > 0 ? c->nsalt : c->nsalt - 1;
    const double I = 2.0 * log(a.G.volume / (a.G.lambda3 * (double)(n_small + 1)));
    const double lnR = move > 0 ? -a.G.beta * dH + a.G.beta_mu + I : -a.G.beta * dH - a.G.beta_mu - I;
    r->dH = dH; r->dU = c->U1 - c->U0; r->dK = c->K1 - c->K0;
    r->H0 = H0; r->H1 = H1;
    r->W_prot = c->Wf[0] + c->Wf[1];
    r->E_switch = c->Esw[0] + c->Esw[1] + c->Esw_pair;
    r->dM = move > 0 ? dH - I / a.G.beta : -dH - I / a.G.beta;
    r->ln_ratio = lnR;
    int acc = 0;
    if (!isfinite(dH)) r->flags |= 2u;   // H4D_FLAG_NONFINITE
    else acc = r->ln_u < lnR;
    if (c->retry) acc = 0;
    r->accepted = acc;
    c->accepted = acc;
}

// Commit or roll back (data).  Accepted insertion: the ghosts become
// physical; accepted deletion: stable compaction without the pair;
// rejection: restore the snapshot.  The canonical state ends in buffer 0.
__global__ __launch_bounds__(kBlock) void k_commit(KArgs a) {
    const Ctl *c = a.ctl;
    const int move = c->move;
    if (move == 0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int bf = c->nf & 1;
    if (c->accepted && move > 0) {
        if (i < c->n_all) {
            const double4 p = a.pos[bf][i];
            a.pos[0][i] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
        }
    } else if (c->accepted && move < 0) {
        const int ic = c->ic, ia = c->ia;
        if (i < c->n_all && i != ic && i != ia) {
            const int d = i - (i > ic) - (i > ia);
            a.tpos[d] = a.pos[bf][i];
            a.ttag[d] = a.tag[i];
            a.ttype[d] = a.type[i];
            a.tmol[d] = a.mol[i];
        }
    } else {
        if (i < c->n) {
            const double4 p = a.pos0[i];
            a.pos[0][i] = with_meta(p.x, p.y, p.z, meta_of(p) & ~kFlyBit);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_commit2(KArgs a) {
    const Ctl *c = a.ctl;
    if (!(c->accepted && c->move < 0)) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < c->n_all - 2) {
        a.pos[0][i] = a.tpos[i];
        a.tag[i] = a.ttag[i];
        a.type[i] = a.ttype[i];
        a.mol[i] = a.tmol[i];
    }
}

__global__ void k_commit_ctl(KArgs a) {
    Ctl *c = a.ctl;
    TrialRec *r = a.rec;
    if (c->accepted) {
        if (c->move > 0) { c->n += 2; c->nsalt += 1; c->next_tag += 2; }
        else { c->n -= 2; c->nsalt -= 1; }
    }
    c->n_all = c->n;
    r->n_salt_after = c->nsalt;
    if (!c->retry) c->trial += 1;
}

// Sum of list lengths of the current state (for the roofline byte count).
__global__ __launch_bounds__(kBlock) void k_sum_nbr(KArgs a, unsigned long long *out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    unsigned long long v = (i < a.ctl->n_all) ? (unsigned long long)a.nnbr[i] : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x % kWave) == 0) atomicAdd(out, v);
}

}  // namespace h4d
