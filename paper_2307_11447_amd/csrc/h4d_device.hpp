// h4d_device.hpp -- device-side building blocks of the H4D library (gfx950).
//
// Counter-based random numbers, the pair potentials at the 4D distance, the
// altitude schedule and wavefront reductions.  Included by the kernels only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace h4d {

constexpr int kMaxTypes = 8;
constexpr int kBlock = 256;          // threads per block of the atom kernels
constexpr int kWave = 64;            // gfx950 wavefront

// meta word of an atom (packed next to its coordinates): type and flags
constexpr int kTypeMask = 0xF;
constexpr int kFlyBit = 0x10;
constexpr int kFastBit = 0x20;       // moved beyond half the skin since the list build
constexpr int kMolBit = 0x40;        // belongs to a rigid 3-site water
constexpr int kFastCap = 256;        // capacity of the fast-atom list

// error bits of the control block
constexpr unsigned kErrNbr = 0x1u;    // neighbour list capacity exceeded
constexpr unsigned kErrCell = 0x2u;   // cell capacity exceeded
constexpr unsigned kErrSkin = 0x4u;   // an atom moved more than skin/2 before a rebuild
constexpr unsigned kErrCap = 0x8u;    // atom capacity exceeded
constexpr unsigned kErrFast = 0x10u;  // fast-atom list full
constexpr unsigned kErrNonfinite = 0x20u;  // a position became non-finite or left the box (the trajectory blew up)

// purposes of the counter-based generator
constexpr uint64_t kPurposeSelect = 1, kPurposeMB = 2, kPurposeNsteps = 3, kPurposeBias = 6;
constexpr uint64_t kPurposeReverse = 7, kPurposeMD = 8, kPurposeRefresh = 9, kPurposeInitV = 10;

// move code of an equilibrium phase (the trials are +1 / -1, 0 idle)
constexpr int kMoveMD = 2;

// --------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with Weyl-sequence key bumps.
// --------------------------------------------------------------------------
struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ u64x4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                        uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    u64x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// top 52 bits -> (m + 1/2) 2^-52, strictly inside (0, 1)
__device__ __forceinline__ double unit_open(uint64_t b) {
    return ((double)(b >> 12) + 0.5) * 0x1p-52;
}

// --------------------------------------------------------------------------
// Model constants shared by every box, passed by value to every kernel.
// --------------------------------------------------------------------------
struct Geo {
    double rc_lj2, rc_c2, rc_max2, rlist2, half_skin2;
    float rc_lj2f, rc_c2f, rc_max2f;
    double alpha, alpha2, cex, Sc, erfc_rc_over_rc, rc_coul;   // damped shifted force
    float alphaf, alpha2f, cexf, Scf, erfc_rc_over_rcf, rc_coulf;
    float nalpha2_log2e;     // -alpha^2 log2(e): exp(-alpha^2 s^2) = 2^(nalpha2_log2e s^2)
    float p_alpha;           // 0.3275911 alpha (argument scale of the erfc fit)
    double dt, half_dt, accel, kT, w_max, kappa;
    double lambda3, beta, beta_mu;
    int n_types;
    int water;
    double d_oh, d_hh;
    // rigid water: masses and the canonical triangle about its centre of mass
    // (O at (0, ra), H at (-rc_w, -rb) and (rc_w, -rb))
    double m_o, m_h, ra, rb, rc_w;
    int n_mol;
    // bimodal bias of the flying anion's offset from the cation (Sec. II B 4,
    // Eq. 14); bias_alpha = 0: the uniform placement of Eq. (4)
    double bias_xb, bias_alpha;
    // altitude schedule (see altitude())
    int schedule;
    double schedule_n;
    // momenta: 0 a fresh Maxwell-Boltzmann draw for every trial; 1 the
    // state's own, carried between trials with the two-end reversal
    int momenta;
    double md_refresh;       // equilibrium phase: v <- c v + sqrt(1 - c^2) xi
    // species-specific w_max: the anion flies at w_ratio times the cation's
    // altitude (1: both at the same altitude)
    double w_ratio;
    // early rejection: half the edge of the cube V_ex around the flying
    // cation (0: off)
    double v_ex_half;
};

// --------------------------------------------------------------------------
// One periodic box of a batch: its geometry and where its atoms and cells
// live in the shared arrays.  Atom slots [a0, a0 + cap) and cells
// [c0, c0 + nc); a0 and cap are multiples of kBlock, so no block of an atom
// kernel straddles two boxes.
// --------------------------------------------------------------------------
struct Box {
    double L[3];
    double fx_inv[3];        // 2^32 / L: FP64 coordinate -> 32-bit fixed point
    float fx_scale[3];       // L / 2^32
    int ncell[3];
    int use_cells;           // 0: fewer than 3 list cells per edge, all pairs
    int a0, cap;
    int c0, nc;
    double volume;
    uint64_t stream;         // second word of this box's Philox key
    double bias_c[3];        // Eq. (14) normalisation per edge: sqrt(alpha / pi) / (erf - erf)
};

// per type-pair coefficients, indexed ti * kMaxTypes + tj
struct PairCoef {
    double sig2, eps, qqk, lj_shift;     // lj_shift = (s/rc)^12 - (s/rc)^6
    float sig2f, eps24f, qqkf, lj_shiftf;
};

// --------------------------------------------------------------------------
// Altitude schedule, Eq. (2): constant vertical velocity.
// --------------------------------------------------------------------------
// Altitude of the flyers before step k of nf.  An insertion runs the
// schedule forwards from w_max to 0, a deletion backwards (j = nf - k), so
// each is the time reversal of the other.  schedule 0: constant vertical
// velocity (Eq. 2); 1: w_max (1 - x^n) and 2: w_max (1 - x)^n, x = j / nf
// (the two variable-velocity schedules of the supplement; n = 1 gives
// Eq. 2 again).
__device__ __forceinline__ double altitude(const Geo &G, int move, int k, int nf) {
    if (nf <= 0) return 0.0;   // an instantaneous exchange switches at once
    const int j = move > 0 ? k : nf - k;
    if (G.schedule == 0) return G.w_max * (double)(nf - j) / (double)nf;
    const double x = (double)j / (double)nf;
    return G.w_max * (G.schedule == 1 ? 1.0 - pow(x, G.schedule_n) : pow(1.0 - x, G.schedule_n));
}

// Periodic wrap into [0, L) of a coordinate less than one box edge outside
// it (atoms move far less than L per step); exact, no division.
__device__ __forceinline__ double wrap_coord(double x, double L) {
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
    return x;
}

// Minimum image of a difference of two wrapped coordinates (|d| < L).
__device__ __forceinline__ double min_image(double d, double L) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

__device__ __forceinline__ uint32_t to_fixed(double x, double fx_inv) {
    return (uint32_t)(unsigned long long)(x * fx_inv);
}

__device__ __forceinline__ int meta_of(const double4 &p) {
    return (int)__double_as_longlong(p.w);
}

__device__ __forceinline__ double4 with_meta(double x, double y, double z, int meta) {
    return make_double4(x, y, z, __longlong_as_double((long long)meta));
}

// --------------------------------------------------------------------------
// erfc in FP32 from Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7), sharing
// exp(-x^2) with the force term.
// --------------------------------------------------------------------------
__device__ __forceinline__ float erfc_as(float x, float ex) {
    const float t = __frcp_rn(1.0f + 0.3275911f * x);
    const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f +
                       t * (-1.453152027f + t * 1.061405429f))));
    return poly * ex;
}

// FP32 force coefficients of a non-flying atom of one type against a
// partner with meta bits tj | fly | fast: the flyer's squared altitude w2
// and its Eq. 11 screening folded into qqk, so that the pair loop needs no
// flyer test; a fast partner (its pairs come from the fast list) and the
// null record that pads the lists get no force (zero coefficients at
// w2 = 1e30, far beyond every cutoff), so the loop needs no validity test
// either.  Built per block and step.
struct ForceCoef {
    float lj12, lj6;   // 48 eps sigma^12 and 24 eps sigma^6: f_LJ = (lj12 / s^6 - lj6) / s^8
    float qqk, w2;
};
constexpr int kForceRow = 64;   // partner indices: meta & (kTypeMask | kFlyBit | kFastBit)
constexpr float kFarW2 = 1.0e30f;

// Radial force over distance, -(du/ds)/s, of one pair at squared 4D
// distance s2 (FP32), without branches (both cutoffs by select), with the
// hardware reciprocal square root and exp2 and one reciprocal.  s2 must be
// positive.
__device__ __forceinline__ float pair_fs_f32(const Geo &G, const ForceCoef &c, float s2) {
    const float rs = __builtin_amdgcn_rsqf(s2);
    const float inv = rs * rs;                   // 1 / s^2 without a second transcendental
    const float inv3 = inv * inv * inv;
    const float flj = inv3 * (c.lj12 * inv3 - c.lj6) * inv;
    const float s = s2 * rs;
    const float ex = __builtin_amdgcn_exp2f(G.nalpha2_log2e * s2);
    const float t = __builtin_amdgcn_rcpf(1.0f + G.p_alpha * s);
    const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f +
                       t * (-1.453152027f + t * 1.061405429f))));
    const float fc = c.qqk * ((poly * inv + G.cexf * rs) * ex - G.Scf) * rs;
    return (s2 < G.rc_lj2f ? flj : 0.0f) + (s2 < G.rc_c2f ? fc : 0.0f);
}

// Same in FP64 with the library erfc.
__device__ __forceinline__ double pair_fs_f64(const Geo &G, const PairCoef &c, double s2, double g) {
    double fs = 0.0;
    const double inv = 1.0 / s2;
    if (s2 < G.rc_lj2) {
        const double sr2 = c.sig2 * inv;
        const double sr6 = sr2 * sr2 * sr2;
        fs += 24.0 * c.eps * sr6 * (2.0 * sr6 - 1.0) * inv;
    }
    if (s2 < G.rc_c2) {
        const double s = sqrt(s2);
        const double ex = exp(-G.alpha2 * s2);
        fs += g * c.qqk * (erfc(G.alpha * s) * inv + G.cex * ex / s - G.Sc) / s;
    }
    return fs;
}

// FP32 pair energy (LJ plus screened Coulomb), for accumulation in FP64.
__device__ __forceinline__ float pair_u_f32(const Geo &G, const PairCoef &c, float s2, float g) {
    float u = 0.0f;
    if (s2 < G.rc_lj2f) {
        const float sr2 = c.sig2f * __frcp_rn(s2);
        const float sr6 = sr2 * sr2 * sr2;
        u += c.eps24f * (1.0f / 6.0f) * (sr6 * sr6 - sr6 - c.lj_shiftf);
    }
    if (s2 < G.rc_c2f) {
        const float rs = __frsqrt_rn(s2);
        const float s = s2 * rs;
        const float ec = erfc_as(G.alphaf * s, __expf(-G.alpha2f * s2));
        u += g * c.qqkf * (ec * rs - G.erfc_rc_over_rcf + G.Scf * (s - G.rc_coulf));
    }
    return u;
}

// FP64 pair energies (LJ and Coulomb parts) and -(du/ds)/s.
__device__ __forceinline__ void pair_u_f64(const Geo &G, const PairCoef &c, double s2, double g,
                                           double &ulj, double &uc, double &fs) {
    ulj = 0.0; uc = 0.0; fs = 0.0;
    const double inv = 1.0 / s2;
    if (s2 < G.rc_lj2) {
        const double sr2 = c.sig2 * inv;
        const double sr6 = sr2 * sr2 * sr2;
        ulj = 4.0 * c.eps * (sr6 * sr6 - sr6 - c.lj_shift);
        fs += 24.0 * c.eps * sr6 * (2.0 * sr6 - 1.0) * inv;
    }
    if (s2 < G.rc_c2) {
        const double s = sqrt(s2);
        const double ex = exp(-G.alpha2 * s2);
        const double ec = erfc(G.alpha * s);
        uc = g * c.qqk * (ec / s - G.erfc_rc_over_rc + G.Sc * (s - G.rc_coul));
        fs += g * c.qqk * (ec * inv + G.cex * ex / s - G.Sc) / s;
    }
}

// --------------------------------------------------------------------------
// Wavefront reductions (fixed butterfly order: bitwise reproducible).
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

}  // namespace h4d
