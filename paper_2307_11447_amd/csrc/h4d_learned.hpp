// h4d_learned.hpp -- learned insertion proposal on gfx950.
//
// Multiple-try form of the uniform pair insertion of Eq. (4): an insertion
// draws k uniform candidate pair sites, gives each the log weight
// scale min(s, cap), s the network's logit of the site's 64 features on the
// state before the trajectory, and flies the pair in at one chosen with
// probability proportional to its weight; the Metropolis ratio gains
// ln(W/k) - (log weight of the chosen site), W the sum of the weights.  A
// deletion weighs the removed pair's site and k - 1 fresh candidates on the
// state after its trajectory (pair removed) and gains (log weight of the
// removed site) - ln(W/k).  This is a bias on the initial positions of the
// flying ions, the kind the paper leaves unimplemented (Sec. II B 1), with
// the ratio correction in the Rosenbluth form of its distance bias
// (Sec. II B 4, Eqs. 15-16).  Exact for any weights; k = 1, scale 0 or
// equal weights is the uniform proposal.
//
// Features are summed in 64-bit fixed point (each FP32 term rounded to a
// fixed grid), so a site's features -- and its weight -- do not depend on
// the order of the atoms in memory: the forward and the reverse move see the
// same function of the configuration.
//
// The network, 64 -> 128 -> 128 -> 128 -> 1 with the tanh form of GELU,
// infers in BF16 on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// accumulation) and trains in FP32 (forward, backpropagation, Adam).
#pragma once
#include "h4d_kernels.hpp"

namespace h4d {

constexpr int kFeat = 64, kHid = 128;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kFeat * kHid, kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid,
              kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kHid, kOffW4 = kOffB3 + kHid, kOffB4 = kOffW4 + kHid;
constexpr int kParams = kOffB4 + 1;                     // 41,473
constexpr int kFragL1 = kFeat * kHid / 4, kFragL2 = kHid * kHid / 4;   // bf16x4 fragments per layer
constexpr uint64_t kPurposeCand = 4, kPurposePick = 5;
constexpr double kShellScale = 4294967296.0;            // 2^32: shell-count terms in [0, 1]
constexpr double kEnergyScale = 1048576.0;              // 2^20: beta-scaled terms, clipped to 1e6
constexpr float kTermClip = 1.0e6f;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct LearnArgs {
    int k;                  // candidates per move and box
    int use_net;            // 0: every logit is 0 (equal weights)
    double cap;             // log weight = scale * min(logit, cap)
    double scale;
    // box b's candidate j is row g = b k + j of the candidate arrays
    double *sites;          // (boxes x k) x 6: cation xyz, anion xyz
    float *feat;            // (boxes x k) x 64
    float *logit;           // boxes x k
    float *last_feat;       // boxes x 64: features of each box's inserted / removed pair's site
    const float *theta;     // FP32 parameters
    const bf16x4 *wfrag;    // hidden layers in MFMA fragment order (BF16)
};

// Does box bi take part in the learned step of this phase (0: an insertion
// before its trajectory; 1: a deletion after it)?
__device__ __forceinline__ bool learned_phase(const Ctl *c, int phase) {
    return phase == 0 ? c->move == 1 : c->move == -1;
}

__device__ __forceinline__ float gelu_f(float x) {
    return 0.5f * x * (1.0f + tanhf(0.7978845608028654f * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    const float t = tanhf(0.7978845608028654f * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * 0.7978845608028654f * (1.0f + 3.0f * 0.044715f * x * x);
}

// FP32 -> BF16, round to nearest even
__device__ __forceinline__ short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ float clipf(float v) { return fminf(kTermClip, fmaxf(-kTermClip, v)); }

__device__ __forceinline__ long long to_fix(float v, double scale) { return __double2ll_rn((double)v * scale); }

// FP32 pair parts at squared distance s2: LJ energy, screened DSF energy and
// the Coulomb radial force over distance, -(d uc / ds) / s.
__device__ __forceinline__ void pair_parts_f32(const Geo &G, const PairCoef &c, float s2, float g, float &ulj,
                                               float &uc, float &fcs) {
    ulj = 0.0f; uc = 0.0f; fcs = 0.0f;
    if (s2 < G.rc_lj2f) {
        const float sr2 = c.sig2f / s2;
        const float sr6 = sr2 * sr2 * sr2;
        ulj = c.eps24f * (1.0f / 6.0f) * (sr6 * sr6 - sr6 - c.lj_shiftf);
    }
    if (s2 < G.rc_c2f) {
        const float s = sqrtf(s2);
        const float ex = expf(-G.alpha2f * s2);
        const float ec = erfc_as(G.alphaf * s, ex);
        uc = g * c.qqkf * (ec / s - G.erfc_rc_over_rcf + G.Scf * (s - G.rc_coulf));
        fcs = g * c.qqkf * (ec / s2 + G.cexf * ex / s - G.Scf) / s;
    }
}

// --------------------------------------------------------------------------
// Candidate sites, one thread per (box, candidate).  phase 0 (insertion,
// before the trajectory): candidates j = 0..k-1 from the box's counters
// (t, 4, j, 0 / 1).  phase 1 (deletion, after it): site 0 is the removed
// pair (fixed in 3D), sites 1..k-1 the candidates 0..k-2.
// --------------------------------------------------------------------------
__global__ void k_cand_sites(KArgs a, LearnArgs l, int phase) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nbox * l.k) return;
    const int bi = g / l.k, j = g - bi * l.k;
    const Ctl *c = a.ctl + bi;
    if (!learned_phase(c, phase)) return;
    const Box &B = a.box[bi];
    double *st = l.sites + 6 * (size_t)g;
    if (phase == 1 && j == 0) {
        const int bf = buf_of(-1, c);
        const double4 pc = a.pos[bf][c->wic], pa = a.pos[bf][c->wia];
        st[0] = pc.x; st[1] = pc.y; st[2] = pc.z;
        st[3] = pa.x; st[4] = pa.y; st[5] = pa.z;
        return;
    }
    const uint64_t q = (uint64_t)(phase == 0 ? j : j - 1);
    const u64x4 r0 = philox((uint64_t)c->trial, kPurposeCand, q, 0, a.seed, B.stream);
    const u64x4 r1 = philox((uint64_t)c->trial, kPurposeCand, q, 1, a.seed, B.stream);
    for (int d = 0; d < 3; ++d) {
        st[d] = wrap_coord(B.L[d] * unit_open(r0.v[d]), B.L[d]);
        st[3 + d] = wrap_coord(B.L[d] * unit_open(r1.v[d]), B.L[d]);
    }
}

// --------------------------------------------------------------------------
// Features of the candidate sites, one wavefront per (site, ion), from the
// non-flying atoms of working buffer b listed in cell buffer cb.  Per ion:
// 0.1 x Gaussian shell counts of types 0..3 (six shells of width rc/6 up to
// rc = max cutoff, each term tapered by (1 - r^2/rc^2)^2), asinh of beta U_C, beta |F_C|, beta U_LJ at w = 0, beta
// U_LJ and beta exp(-kappa w_max) U_C at w = w_max, and the nearest atom and
// counter-ion distances over rc (capped at 1).  Pair: separation over rc
// (capped) and asinh(beta u) of the pair itself.  Pair terms are scaled by
// beta, clipped to +-1e6 and summed in fixed point.
// --------------------------------------------------------------------------
__device__ __forceinline__ void site_features(const KArgs &a, const LearnArgs &l, int phase, int b0, int cb) {
    const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) / kWave), lane = threadIdx.x % kWave;
    const int j = wave >> 1, ion = wave & 1;   // j: row of (box, candidate)
    if (j >= a.nbox * l.k) return;
    const int bi = j / l.k;
    const Ctl *c = a.ctl + bi;
    if (phase >= 0 && !learned_phase(c, phase)) return;
    const Box &B = a.box[bi];
    const Geo &G = a.G;
    const int b = buf_of(b0, c);
    const double *st = l.sites + 6 * (size_t)j + 3 * ion;
    const int T = ion ? a.anion_type : a.cation_type, counter = ion ? a.cation_type : a.anion_type;
    const uint4 qs = fixed_of(B, st[0], st[1], st[2], 0);
    const float rc = sqrtf(G.rc_max2f), delta = rc / 6.0f, sd = delta / 2.0f;
    const float beta = (float)G.beta, wmax2 = (float)(G.w_max * G.w_max);
    const float gmax = (float)exp(-G.kappa * G.w_max);
    const PairCoef *crow = a.coef + T * kMaxTypes;
    long long sh[24];
#pragma unroll
    for (int q = 0; q < 24; ++q) sh[q] = 0;
    long long uc0 = 0, ulj0 = 0, uljw = 0, ucw = 0, fx = 0, fy = 0, fz = 0;
    float dmin = INFINITY, dct = INFINITY;
    auto visit = [&](int w) {
        const uint4 q = a.fx[b][w];
        if (q.w & kFlyBit) return;
        const float dx = (float)(int)(qs.x - q.x) * B.fx_scale[0];
        const float dy = (float)(int)(qs.y - q.y) * B.fx_scale[1];
        const float dz = (float)(int)(qs.z - q.z) * B.fx_scale[2];
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rr = sqrtf(r2);
        const int tj = (int)q.w & kTypeMask;
        dmin = fminf(dmin, rr);
        if (tj == counter) dct = fminf(dct, rr);
        if (r2 < G.rc_max2f) {
            const float x = 1.0f - r2 / G.rc_max2f, taper = x * x;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const float z = (rr - ((float)m + 0.5f) * delta) / sd;
                const long long v = to_fix(expf(-0.5f * z * z) * taper, kShellScale);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) sh[6 * tt + m] += (tj == tt) ? v : 0ll;
            }
        }
        float ulj, uc, fcs;
        pair_parts_f32(G, crow[tj], r2, 1.0f, ulj, uc, fcs);
        ulj0 += to_fix(clipf(beta * ulj), kEnergyScale);
        uc0 += to_fix(clipf(beta * uc), kEnergyScale);
        const float fr = clipf(beta * fcs * rr);          // radial Coulomb force
        fx += to_fix(fr * dx / rr, kEnergyScale);
        fy += to_fix(fr * dy / rr, kEnergyScale);
        fz += to_fix(fr * dz / rr, kEnergyScale);
        pair_parts_f32(G, crow[tj], r2 + wmax2, gmax, ulj, uc, fcs);
        uljw += to_fix(clipf(beta * ulj), kEnergyScale);
        ucw += to_fix(clipf(beta * uc), kEnergyScale);
    };
    if (B.use_cells) {
        const double4 ps = make_double4(st[0], st[1], st[2], 0.0);
        const int cx = cell_coord(ps.x, B.L[0], B.ncell[0]);
        const int cy = cell_coord(ps.y, B.L[1], B.ncell[1]);
        const int cz = cell_coord(ps.z, B.L[2], B.ncell[2]);
        for (int t = 0; t < 27; ++t) {
            const int c2 = stencil_cell(B, cx, cy, cz, t);
            const int m = min(a.cell_cnt[cb][c2], a.cell_cap);
            const int *row = a.cell_atoms[cb] + (size_t)c2 * a.cell_cap;
            for (int u = lane; u < m; u += kWave) visit(row[u]);
        }
    } else {
        for (int w = B.a0 + lane; w < B.a0 + c->n_all; w += kWave) visit(w);
    }
    // order-independent reductions: integer sums and minima
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 24; ++q) sh[q] += __shfl_xor(sh[q], off, kWave);
        uc0 += __shfl_xor(uc0, off, kWave);
        ulj0 += __shfl_xor(ulj0, off, kWave);
        uljw += __shfl_xor(uljw, off, kWave);
        ucw += __shfl_xor(ucw, off, kWave);
        fx += __shfl_xor(fx, off, kWave);
        fy += __shfl_xor(fy, off, kWave);
        fz += __shfl_xor(fz, off, kWave);
        dmin = fminf(dmin, __shfl_xor(dmin, off, kWave));
        dct = fminf(dct, __shfl_xor(dct, off, kWave));
    }
    if (lane != 0) return;
    float *out = l.feat + 64 * (size_t)j + 31 * ion;
#pragma unroll
    for (int q = 0; q < 24; ++q) out[q] = (float)(0.1 * ((double)sh[q] / kShellScale));
    const double fxd = (double)fx / kEnergyScale, fyd = (double)fy / kEnergyScale, fzd = (double)fz / kEnergyScale;
    out[24] = (float)asinh((double)uc0 / kEnergyScale);
    out[25] = (float)asinh(sqrt(fxd * fxd + fyd * fyd + fzd * fzd));
    out[26] = (float)asinh((double)ulj0 / kEnergyScale);
    out[27] = (float)asinh((double)uljw / kEnergyScale);
    out[28] = (float)asinh((double)ucw / kEnergyScale);
    out[29] = fminf(dmin, rc) / rc;
    out[30] = fminf(dct, rc) / rc;
    if (ion == 0) {   // the pair's own features
        const double *sa = l.sites + 6 * (size_t)j + 3;
        const uint4 qa = fixed_of(B, sa[0], sa[1], sa[2], 0);
        const float dx = (float)(int)(qs.x - qa.x) * B.fx_scale[0];
        const float dy = (float)(int)(qs.y - qa.y) * B.fx_scale[1];
        const float dz = (float)(int)(qs.z - qa.z) * B.fx_scale[2];
        const float r2 = dx * dx + dy * dy + dz * dz;
        float ulj, uc, fcs;
        pair_parts_f32(G, crow[a.anion_type], r2, 1.0f, ulj, uc, fcs);
        float *pf = l.feat + 64 * (size_t)j;
        pf[62] = fminf(sqrtf(r2), rc) / rc;
        pf[63] = asinhf(clipf(beta * (ulj + uc)));
    }
}

__global__ __launch_bounds__(kBlock) void k_site_features(KArgs a, LearnArgs l, int phase, int b0, int cb) {
    site_features(a, l, phase, b0, cb);
}

// test hook (one box): features of given sites on the state sorted into
// working buffer 0 / cell buffer 0 (h4d_build_neighbors)
__global__ __launch_bounds__(kBlock) void k_site_features_hook(KArgs a, LearnArgs l) { site_features(a, l, -1, 0, 0); }

// --------------------------------------------------------------------------
// Network inference in BF16 on the matrix cores.  One block of four
// wavefronts per 64 sites; wavefront w owns rows 16w..16w+15.  For
// v_mfma_f32_16x16x16_bf16 lane l holds A[l % 16][4 (l / 16) + v],
// B[4 (l / 16) + v][l % 16] and D[4 (l / 16) + v][l % 16], v = 0..3.
// Activations stay in LDS (BF16); the output layer is a FP32 dot product
// reduced over the 16 lanes of each row group in a fixed order.
// --------------------------------------------------------------------------
__device__ __forceinline__ void mlp_tile(const float *feat, int n, const float *theta, const bf16x4 *wfrag,
                                         float *out) {
    __shared__ short xbuf[2][64][kHid + 8];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int row0 = blockIdx.x * 64;
    const int i16 = lane % 16, g4 = lane / 16;
    for (int q = lane; q < 16 * kFeat; q += kWave) {
        const int r = q / kFeat, cidx = q % kFeat;
        const int gr = row0 + 16 * wave + r;
        xbuf[0][16 * wave + r][cidx] = to_bf16(gr < n ? feat[(size_t)gr * kFeat + cidx] : 0.0f);
    }
    __syncthreads();
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int layer = 0; layer < 3; ++layer) {
        const int K = layer == 0 ? kFeat : kHid;
        const int in = layer & 1, ob = in ^ 1;
        const bf16x4 *wf = wfrag + (layer == 0 ? 0 : (layer == 1 ? kFragL1 : kFragL1 + kFragL2));
        const float *bias = theta + (layer == 0 ? kOffB1 : (layer == 1 ? kOffB2 : kOffB3));
        for (int nt = 0; nt < kHid / 16; ++nt) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kk = 0; kk < K / 16; ++kk) {
                bf16x4 av;
#pragma unroll
                for (int v = 0; v < 4; ++v) av[v] = xbuf[in][16 * wave + i16][16 * kk + 4 * g4 + v];
                const bf16x4 bv = wf[((size_t)nt * (K / 16) + kk) * kWave + lane];
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
            }
            const int col = 16 * nt + i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float h = gelu_f(acc[v] + bias[col]);
                if (layer < 2) xbuf[ob][16 * wave + 4 * g4 + v][col] = to_bf16(h);
                else part[v] += h * theta[kOffW4 + col];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
        for (int off = 8; off > 0; off >>= 1) part[v] += __shfl_xor(part[v], off, 16);
    if (i16 == 0)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gr = row0 + 16 * wave + 4 * g4 + v;
            if (gr < n) out[gr] = part[v] + theta[kOffB4];
        }
}

__global__ __launch_bounds__(256) void k_mlp_infer(const float *feat, int n, const float *theta, const bf16x4 *wfrag,
                                                   float *out) {
    mlp_tile(feat, n, theta, wfrag, out);
}

// BF16 fragments of the three hidden layers: fragment (nt, kk, lane) holds
// W[16 kk + 4 (lane / 16) + v][16 nt + lane % 16], v = 0..3.
__global__ void k_mlp_pack(const float *theta, bf16x4 *wfrag) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= kFragL1 + 2 * kFragL2) return;
    int layer, q;
    if (f < kFragL1) { layer = 0; q = f; }
    else if (f < kFragL1 + kFragL2) { layer = 1; q = f - kFragL1; }
    else { layer = 2; q = f - kFragL1 - kFragL2; }
    const int K = layer == 0 ? kFeat : kHid;
    const int off = layer == 0 ? kOffW1 : (layer == 1 ? kOffW2 : kOffW3);
    const int lane = q % kWave, kk = (q / kWave) % (K / 16), nt = q / kWave / (K / 16);
    bf16x4 v4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int k = 16 * kk + 4 * (lane / 16) + v, j = 16 * nt + lane % 16;
        v4[v] = to_bf16(theta[off + k * kHid + j]);
    }
    wfrag[f] = v4;
}

__global__ void k_zero_logits(KArgs a, LearnArgs l, int phase) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.nbox * l.k || !learned_phase(a.ctl + g / l.k, phase)) return;
    l.logit[g] = 0.0f;
}

// logits of every box's candidates (after k_site_features): one pass over
// the boxes x k rows; a 64-row tile whose boxes all sit out this phase
// returns at once
__global__ __launch_bounds__(256) void k_mlp_infer_move(KArgs a, LearnArgs l, int phase) {
    const int rows = a.nbox * l.k, row0 = blockIdx.x * 64;
    const int b_lo = row0 / l.k, b_hi = min(row0 + 63, rows - 1) / l.k;
    bool any = false;
    for (int bi = b_lo; bi <= b_hi; ++bi) any |= learned_phase(a.ctl + bi, phase);
    if (!any) return;
    mlp_tile(l.feat, rows, l.theta, l.wfrag, l.logit);
}

// --------------------------------------------------------------------------
// The multiple-try step, one block per box, FP64, with log weights
// lw = scale min(s, cap) taken relative to the largest.  Thread t sums the
// weights of a contiguous chunk of candidates in order; thread 0 adds the
// chunks in order (a fixed order for a given k).  Insertion: the first
// candidate whose running weight exceeds u W (uniform (t, 5, 0, 0)); the
// ghosts move to it; ln q = ln(W/k) - lw(chosen).  Deletion: ln q =
// lw(removed) - ln(W/k).
// --------------------------------------------------------------------------
constexpr int kMtmBlock = 256;

__global__ __launch_bounds__(kMtmBlock) void k_mtm_select(KArgs a, LearnArgs l, int phase) {
    const int bi = blockIdx.x, tid = threadIdx.x;
    Ctl *c = a.ctl + bi;
    if (!learned_phase(c, phase)) return;
    const int k = l.k;
    const size_t g0 = (size_t)bi * k;
    __shared__ double s_part[kMtmBlock];
    __shared__ double s_mx, s_lnWk;
    __shared__ int s_sel;
    auto lw = [&](int j) { return l.scale * fmin((double)l.logit[g0 + j], l.cap); };
    const int chunk = (k + kMtmBlock - 1) / kMtmBlock;
    const int lo = min(k, tid * chunk), hi = min(k, lo + chunk);
    double mx = -INFINITY;
    for (int j = lo; j < hi; ++j) mx = fmax(mx, lw(j));
    s_part[tid] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = s_part[0];
        for (int q = 1; q < kMtmBlock; ++q) m = fmax(m, s_part[q]);
        s_mx = m;
    }
    __syncthreads();
    mx = s_mx;
    double acc = 0.0;
    for (int j = lo; j < hi; ++j) acc += exp(lw(j) - mx);
    __syncthreads();
    s_part[tid] = acc;
    __syncthreads();
    if (tid == 0) {
        double W = 0.0;
        for (int q = 0; q < kMtmBlock; ++q) W += s_part[q];
        const double lnWk = mx + log(W) - log((double)k);
        s_lnWk = lnWk;
        int sel = 0;
        if (phase == 0) {
            const Box &B = a.box[bi];
            const u64x4 r = philox((uint64_t)c->trial, kPurposePick, 0, 0, a.seed, B.stream);
            const double target = unit_open(r.v[0]) * W;
            double run = 0.0;
            int q = 0;
            while (q < kMtmBlock - 1 && run + s_part[q] <= target) run += s_part[q++];
            sel = min(k, q * chunk + chunk) - 1;   // rounding at the chunk's end: its last candidate
            for (int j = min(k, q * chunk); j < min(k, q * chunk + chunk); ++j) {
                run += exp(lw(j) - mx);
                if (run > target) { sel = j; break; }
            }
            c->lnq = lnWk - lw(sel);
            const double *st = l.sites + 6 * (g0 + sel);
            double4 p = a.cpos[c->ic];
            a.cpos[c->ic] = with_meta(st[0], st[1], st[2], meta_of(p));
            p = a.cpos[c->ia];
            a.cpos[c->ia] = with_meta(st[3], st[4], st[5], meta_of(p));
        } else {
            c->lnq = lw(0) - lnWk;
        }
        s_sel = sel;
    }
    __syncthreads();
    if (tid < kFeat) l.last_feat[(size_t)kFeat * bi + tid] = l.feat[kFeat * (g0 + s_sel) + tid];
}

// ==========================================================================
// FP32 training: dense layers, mean-squared loss, backpropagation, Adam.
// Every reduction runs in a fixed order (no atomics).
// ==========================================================================
// Z = X W + b, A = gelu(Z) (act) or Z; X n x I, W I x O (row-major)
// (Z may be null: the forward alone keeps only the activations)
__global__ void k_dense_fwd(const float *X, const float *W, const float *b, float *Z, float *A, int n, int I, int O,
                            int act) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * O) return;
    const int r = idx / O, o = idx % O;
    float z = b[o];
    for (int i = 0; i < I; ++i) z += X[(size_t)r * I + i] * W[(size_t)i * O + o];
    if (Z) Z[idx] = z;
    A[idx] = act ? gelu_f(z) : z;
}

// one block: dS = 2 (s - t) / n and the mean-squared loss
__global__ __launch_bounds__(256) void k_mse(const float *s, const float *t, int n, float *dS, float *loss) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (int r = threadIdx.x; r < n; r += 256) {
        const float d = s[r] - t[r];
        dS[r] = 2.0f * d / (float)n;
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

// gW[i][o] = sum_r X[r][i] dZ[r][o]; gb[o] = sum_r dZ[r][o]
__global__ void k_wgrad(const float *X, const float *dZ, int n, int I, int O, float *gW, float *gb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (I + 1) * O) return;
    const int i = idx / O, o = idx % O;
    float acc = 0.0f;
    if (i < I) {
        for (int r = 0; r < n; ++r) acc += X[(size_t)r * I + i] * dZ[(size_t)r * O + o];
        gW[(size_t)i * O + o] = acc;
    } else {
        for (int r = 0; r < n; ++r) acc += dZ[(size_t)r * O + o];
        gb[o] = acc;
    }
}

// dZp[r][i] = (sum_o dZ[r][o] W[i][o]) gelu'(Zp[r][i])
__global__ void k_dgrad(const float *dZ, const float *W, const float *Zp, int n, int I, int O, float *dZp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * I) return;
    const int r = idx / I, i = idx % I;
    float acc = 0.0f;
    for (int o = 0; o < O; ++o) acc += dZ[(size_t)r * O + o] * W[(size_t)i * O + o];
    dZp[idx] = acc * gelu_grad_f(Zp[idx]);
}

// Adam (Kingma & Ba) with bias correction factors c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t)
// and decoupled weight decay wd (Loshchilov & Hutter)
__global__ void k_adam(float *theta, float *m, float *v, const float *g, int N, float lr, float b1, float b2, float eps,
                       float c1, float c2, float wd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * theta[i]);
}

// rows idx[0..n) of src (stride 64) and their targets
__global__ void k_gather_rows(const float *src, const float *tsrc, const int *idx, int n, float *dst, float *tdst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * kFeat) return;
    const int r = q / kFeat, c = q % kFeat;
    dst[q] = src[(size_t)idx[r] * kFeat + c];
    if (c == 0) tdst[r] = tsrc[idx[r]];
}

}  // namespace h4d
