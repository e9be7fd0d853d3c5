// h4d_runtime.hip -- host side of the C ABI declared in include/h4d.h.
//
// Owns the device buffers of a system, enqueues the kernels of each trial
// on the caller's stream, and reads back one small record per trial (the
// only synchronisation of a trial).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "h4d.h"
#include "h4d_learned.hpp"
#include <random>

using namespace h4d;

static_assert(sizeof(TrialRec) == sizeof(h4d_trial), "record layout");
static_assert(kMoveMD == H4D_MOVE_MD, "move code of an equilibrium phase");
static_assert(kFlagInstant == H4D_FLAG_INSTANT && kFlagIdle == H4D_FLAG_IDLE, "record flags");

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPC(x)                                                                                   \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return fail(H4D_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

int blocks_for(int n) { return std::max(1, (n + kBlock - 1) / kBlock); }

}  // namespace

struct h4d_system {
    h4d_params p{};
    hipStream_t stream = nullptr;
    KArgs a{};
    PairCoef coef_h[kMaxTypes * kMaxTypes]{};
    int nbox = 1;
    bool cells = true;          // every box has >= 3 list cells per edge
    std::vector<Box> box_h;
    std::vector<int> n_host, nsalt_host;   // per box, after the last round
    int n_mol = 0;
    int rebuild_every = 1;
    int clean_trials = 0;
    bool interval_tuned = false;   // the autotuner fixed the base interval
    bool speculative = false;      // the boxes are replicas of one chain (one Philox key)
    bool vel_canonical = false;    // the state's momenta are the canonical ones (after a phase)
    int list_split = 0;            // list-build blocks per cell (0: automatic)
    int list_units = 8;            // list-build centre units per cell: 8 sub-cells or 1 cell
    double step_bytes_est = 0.0;   // a step's list entries and own state, from the densities at set-up
    int list_loads = -1;           // list-index loads of the FP32 pair pass: -1 by size, 0 cached, 1 non-temporal
    int partial_blocks = 0;
    TrialRec *h_rec = nullptr;  // per box (pinned)
    Ctl *h_ctl = nullptr;       // per box (pinned)
    // step-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int64_t step_launches = 0;
    double step_ms = 0.0;
    double atom_launches = 0.0;   // atoms integrated, summed over the timed step launches
    int trial_rebuilds = 0;
    int64_t retries = 0;
    int64_t retries_total = 0, nonfinite = 0;   // over the handle's life
    int trial_M = 1;            // rebuild interval of the round being run
    int cl = 0;                 // cell buffer of the current list (the next binning uses cl ^ 1)
    // captured round graphs, keyed by launch shape; dropped when buffers move
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int, int, int>, hipGraphExec_t> graphs;
    bool graphs_ok[2] = {true, false};  // timed rounds launch eagerly (events per step kernel)
    std::vector<void *> allocs;
    // running statistics per box (Eq. 1)
    struct Stats {
        int64_t n_trials = 0, n_ins = 0, n_ins_acc = 0, n_del = 0, n_del_acc = 0;
        double N_sum = 0.0, N2_sum = 0.0;
    };
    std::vector<Stats> stats;
    Stats chain;                   // speculative handles: the chain's statistics
    // learned proposal: k candidates per move and box, 0 = uniform
    LearnArgs la{};

    template <class T>
    int alloc(T **ptr, size_t count) {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
            return fail(H4D_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        allocs.push_back(q);
        *ptr = static_cast<T *>(q);
        return H4D_OK;
    }
    void release(void *q) {
        drop_graphs();
        auto it = std::find(allocs.begin(), allocs.end(), q);
        if (it != allocs.end()) { (void)hipFree(q); allocs.erase(it); }
    }
    void drop_graphs() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    ~h4d_system() {
        drop_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (void *q : allocs) (void)hipFree(q);
        if (h_rec) (void)hipHostFree(h_rec);
        if (h_ctl) (void)hipHostFree(h_ctl);
    }
};

namespace {

int check_params(const h4d_params &p) {
    if (p.n_types < 1 || p.n_types > kMaxTypes) return fail(H4D_EINVAL, "n_types must be in [1, 8]");
    if (p.cation_type < 0 || p.cation_type >= p.n_types || p.anion_type < 0 || p.anion_type >= p.n_types ||
        p.cation_type == p.anion_type)
        return fail(H4D_EINVAL, "cation_type / anion_type invalid");
    if (p.n_steps_max > 0) {
        if (p.n_steps_min < 1 || p.n_steps_max < p.n_steps_min)
            return fail(H4D_EINVAL, "need 1 <= n_steps_min <= n_steps_max");
    } else if (p.n_steps < 1) {
        return fail(H4D_EINVAL, "n_steps must be >= 1");
    }
    if (p.lanes_per_atom != 0 && p.lanes_per_atom != 4 && p.lanes_per_atom != 8 && p.lanes_per_atom != 16)
        return fail(H4D_EINVAL, "lanes_per_atom must be 0, 4, 8 or 16");
    if (p.precision != H4D_PREC_FP64 && p.precision != H4D_PREC_FP32)
        return fail(H4D_EINVAL, "precision must be H4D_PREC_FP64 or H4D_PREC_FP32");
    for (int t = 0; t < p.n_types; ++t)
        if (!(p.mass[t] > 0.0)) return fail(H4D_EINVAL, "masses must be positive");
    if (!(p.kT > 0.0) || !(p.dt > 0.0) || !(p.accel > 0.0) || !(p.lambda_s > 0.0))
        return fail(H4D_EINVAL, "kT, dt, accel and lambda_s must be positive");
    if (!(p.rc_lj > 0.0) || !(p.rc_coul > 0.0) || !(p.skin >= 0.0) || !(p.w_max >= 0.0) ||
        !(p.dsf_alpha >= 0.0))
        return fail(H4D_EINVAL, "cutoffs must be positive, skin, w_max and dsf_alpha non-negative");
    if (p.schedule < 0 || p.schedule > 2 || (p.schedule != 0 && !(p.schedule_n >= 1.0 && std::isfinite(p.schedule_n))))
        return fail(H4D_EINVAL, "schedule must be 0, 1 or 2, with schedule_n >= 1 for 1 and 2");
    if (p.momenta != 0 && p.momenta != 1) return fail(H4D_EINVAL, "momenta must be 0 or 1");
    if (!(p.md_refresh >= 0.0 && p.md_refresh <= 1.0)) return fail(H4D_EINVAL, "md_refresh must lie in [0, 1]");
    if (!(p.w_max_ratio >= 0.0 && std::isfinite(p.w_max_ratio)))
        return fail(H4D_EINVAL, "w_max_ratio must be finite and >= 0 (0: the cation's w_max)");
    if (!(p.v_ex_edge >= 0.0 && std::isfinite(p.v_ex_edge))) return fail(H4D_EINVAL, "v_ex_edge must be finite and >= 0");
    if (p.water && !(p.d_oh > 0.0 && p.d_hh > 0.0 && p.d_hh < 2.0 * p.d_oh))
        return fail(H4D_EINVAL, "rigid water needs 0 < d_hh < 2 d_oh");
    return H4D_OK;
}

double rlist_of(const h4d_params &p) { return std::max(p.rc_lj, p.rc_coul) + p.skin; }

void setup_geo(h4d_system *s) {
    const h4d_params &p = s->p;
    Geo &G = s->a.G;
    const double rc = std::max(p.rc_lj, p.rc_coul);
    const double rlist = rlist_of(p);
    G.rc_lj2 = p.rc_lj * p.rc_lj;
    G.rc_c2 = p.rc_coul * p.rc_coul;
    G.rc_max2 = rc * rc;
    G.rlist2 = rlist * rlist;
    G.half_skin2 = 0.25 * p.skin * p.skin;
    G.rc_lj2f = (float)G.rc_lj2;
    G.rc_c2f = (float)G.rc_c2;
    G.rc_max2f = (float)G.rc_max2;
    const double al = p.dsf_alpha, Rc = p.rc_coul;
    const double two_over_sqrtpi = 1.1283791670955125739;
    G.alpha = al;
    G.alpha2 = al * al;
    G.cex = two_over_sqrtpi * al;
    G.erfc_rc_over_rc = std::erfc(al * Rc) / Rc;
    G.Sc = std::erfc(al * Rc) / (Rc * Rc) + two_over_sqrtpi * al * std::exp(-al * al * Rc * Rc) / Rc;
    G.rc_coul = Rc;
    G.alphaf = (float)G.alpha;
    G.alpha2f = (float)G.alpha2;
    G.cexf = (float)G.cex;
    G.Scf = (float)G.Sc;
    G.erfc_rc_over_rcf = (float)G.erfc_rc_over_rc;
    G.nalpha2_log2e = (float)(-al * al * 1.4426950408889634074);
    G.p_alpha = (float)(0.3275911 * al);
    G.rc_coulf = (float)G.rc_coul;
    G.dt = p.dt;
    G.half_dt = 0.5 * p.dt;
    G.accel = p.accel;
    G.kT = p.kT;
    G.w_max = p.w_max;
    G.schedule = p.schedule;
    G.schedule_n = p.schedule_n;
    G.momenta = p.momenta;
    G.md_refresh = p.md_refresh;
    G.w_ratio = p.w_max_ratio > 0.0 ? p.w_max_ratio : 1.0;
    G.v_ex_half = 0.5 * p.v_ex_edge;
    G.kappa = p.kappa_sr;
    G.lambda3 = p.lambda_s * p.lambda_s * p.lambda_s;
    G.beta = 1.0 / p.kT;
    G.beta_mu = p.beta_mu;
    G.n_types = p.n_types;
    G.water = p.water;
    G.d_oh = p.d_oh;
    G.d_hh = p.d_hh;
    // Lorentz-Berthelot pair table
    for (int i = 0; i < kMaxTypes; ++i)
        for (int j = 0; j < kMaxTypes; ++j) {
            PairCoef &c = s->coef_h[i * kMaxTypes + j];
            c = PairCoef{};
            if (i >= p.n_types || j >= p.n_types) continue;
            const double sig = 0.5 * (p.sigma[i] + p.sigma[j]);
            const double eps = std::sqrt(p.eps[i] * p.eps[j]);
            const double a6 = std::pow(sig / p.rc_lj, 6.0);
            c.sig2 = sig * sig;
            c.eps = eps;
            c.qqk = p.coulomb_k * p.charge[i] * p.charge[j];
            c.lj_shift = a6 * a6 - a6;
            c.sig2f = (float)c.sig2;
            c.eps24f = (float)(24.0 * eps);
            c.qqkf = (float)c.qqk;
            c.lj_shiftf = (float)c.lj_shift;
        }
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Bimodal bias (Sec. II B 4): parameters into Geo and the Eq. (14)
// normalisation of every box edge; the Gaussians (6 standard deviations out
// from +-x_b) must fit within half an edge, so that a drawn offset all but
// never has to be redrawn.
int setup_bias(h4d_system *s, double xb, double alpha) {
    if (!(std::isfinite(xb) && std::isfinite(alpha)) || xb < 0.0 || alpha < 0.0)
        return fail(H4D_EINVAL, "bias_xb and bias_alpha must be finite and >= 0");
    if (alpha > 0.0) {
        const double reach = xb + 6.0 / std::sqrt(2.0 * alpha);
        for (const Box &B : s->box_h)
            for (int d = 0; d < 3; ++d)
                if (reach > 0.5 * B.L[d])
                    return fail(H4D_EINVAL, "bias: x_b + 6 / sqrt(2 alpha_b) must not exceed half a box edge");
    }
    s->a.G.bias_xb = alpha > 0.0 ? xb : 0.0;
    s->a.G.bias_alpha = alpha;
    for (Box &B : s->box_h)
        for (int d = 0; d < 3; ++d) {
            const double sa = std::sqrt(alpha);
            B.bias_c[d] = alpha > 0.0 ? std::sqrt(alpha / 3.14159265358979323846) /
                                            (std::erf(sa * (xb + 0.5 * B.L[d])) - std::erf(sa * (xb - 0.5 * B.L[d])))
                                      : 0.0;
        }
    return H4D_OK;
}

// Geometry and placement of every box: slots [a0, a0 + cap), cells [c0, c0 + nc).
int setup_boxes(h4d_system *s, const double *edges, const int32_t *n_atoms) {
    const h4d_params &p = s->p;
    const double rlist = rlist_of(p);
    const double rc = std::max(p.rc_lj, p.rc_coul);
    const double two32 = 4294967296.0;
    s->box_h.assign(s->nbox, Box{});
    int a0 = 0, c0 = 0, n_cells = 0, n_pairs = 0;
    for (int b = 0; b < s->nbox; ++b) {
        Box &B = s->box_h[b];
        const int n = n_atoms[b];
        for (int d = 0; d < 3; ++d) {
            const double L = edges[3 * b + d];
            if (!(L >= 2.0 * rc)) return fail(H4D_EINVAL, "every box edge must be at least twice the largest cutoff");
            B.L[d] = L;
            B.fx_inv[d] = two32 / L;
            B.fx_scale[d] = (float)(L / two32);
            B.ncell[d] = (int)std::floor(L / rlist);
        }
        B.use_cells = B.ncell[0] >= 3 && B.ncell[1] >= 3 && B.ncell[2] >= 3;
        if (!B.use_cells) B.ncell[0] = B.ncell[1] = B.ncell[2] = 1;
        (B.use_cells ? n_cells : n_pairs) += 1;
        int cap = p.capacity > 0 ? p.capacity : n + std::max(1024, n / 8);
        if (cap < n + 2) return fail(H4D_EINVAL, "capacity below n_atoms + 2");
        cap = round_up(cap, kBlock);
        if (!B.use_cells && cap > 8192)
            return fail(H4D_EINVAL, "a box with fewer than 3 list cells per edge is limited to 8192 atoms");
        B.a0 = a0;
        B.cap = cap;
        B.c0 = c0;
        B.nc = B.ncell[0] * B.ncell[1] * B.ncell[2];
        B.volume = B.L[0] * B.L[1] * B.L[2];
        B.stream = p.stream + (s->speculative ? 0u : (uint64_t)b);
        a0 += cap;
        c0 += B.nc;
        if (a0 > (1 << 30)) return fail(H4D_EINVAL, "too many atom slots");
    }
    if (n_cells && n_pairs)
        return fail(H4D_EINVAL, "the boxes of a batch must all have >= 3 list cells per edge, or all fewer");
    s->cells = n_cells > 0;
    s->a.slots = a0;
    s->a.ncell_total = c0;
    s->a.nbox = s->nbox;
    return H4D_OK;
}

// Neighbour and cell capacities from the densest box (grown on overflow).
void initial_capacities(h4d_system *s, const int32_t *n_atoms) {
    const h4d_params &p = s->p;
    const double rlist = rlist_of(p);
    int nbr = 32, cc = 32, capmax = 0;
    s->step_bytes_est = 0.0;
    for (int b = 0; b < s->nbox; ++b) {
        const Box &B = s->box_h[b];
        const double rho = std::max(1.0, (double)n_atoms[b]) / B.volume;
        const double nb = 4.18879020478639 * rlist * rlist * rlist * rho;
        s->step_bytes_est += (double)n_atoms[b] * (4.0 * nb + 160.0);
        nbr = std::max(nbr, std::min((int)(1.5 * nb) + 32, B.cap + kMaxLanes));
        cc = std::max(cc, (int)(1.6 * rho * B.volume / B.nc) + 16);
        capmax = std::max(capmax, B.cap);
    }
    s->a.nbr_cap = round_up(nbr, kMaxLanes);
    s->a.cell_cap = s->cells ? std::min(cc, std::max(32, capmax)) : capmax;
    // list-build blocks per cell: one per sub-cell when a sub-cell holds at
    // least two atoms per wavefront on average, else one per cell
    long long n_all = 0;
    for (int b = 0; b < s->nbox; ++b) n_all += n_atoms[b];
    const double per_cell = s->a.ncell_total > 0 ? (double)n_all / s->a.ncell_total : 0.0;
    s->list_units = per_cell >= 8.0 * 2 * kListWaves ? 8 : 1;
}

size_t nbr_elems(const h4d_system *s) { return (size_t)s->a.slots * (size_t)s->a.nbr_cap; }

// Non-temporal list loads in the FP32 pair pass when a step's streamed data
// (the list entries and the atoms' own state, estimated from the densities
// at set-up) exceeds the 256 MB Infinity Cache: data that fits is re-read
// from it step after step, data that does not only evicts the gathered
// records on its way through (measured: the water box 3 % faster, the 256
// boxes 1 %, the 32k box 12 % slower with them).
bool nt_lists(const h4d_system *s) {
    if (s->list_loads >= 0) return s->list_loads != 0;
    return s->step_bytes_est > 256.0 * 1024 * 1024;
}

int alloc_lists(h4d_system *s) {
    int rc;
    if ((rc = s->alloc(&s->a.nbr, nbr_elems(s)))) return rc;
    for (int q = 0; q < 2; ++q) {
        if ((rc = s->alloc(&s->a.cell_cnt[q], (size_t)s->a.ncell_total))) return rc;
        if ((rc = s->alloc(&s->a.cell_atoms[q], (size_t)s->a.ncell_total * s->a.cell_cap))) return rc;
        HIPC(hipMemset(s->a.cell_cnt[q], 0, sizeof(int) * s->a.ncell_total));
    }
    if ((rc = s->alloc(&s->a.cell_off, (size_t)s->a.ncell_total))) return rc;
    for (int q = 0; q < 2; ++q) {
        if ((rc = s->alloc(&s->a.cell_sub[q], 8 * (size_t)s->a.ncell_total))) return rc;
        HIPC(hipMemset(s->a.cell_sub[q], 0, sizeof(int) * 8 * s->a.ncell_total));
    }
    if ((rc = s->alloc(&s->a.slot_sub, (size_t)s->a.slots))) return rc;
    HIPC(hipMemset(s->a.slot_sub, 0, sizeof(int) * s->a.slots));
    if ((rc = s->alloc(&s->a.fast, (size_t)s->nbox * 3 * kFastCap))) return rc;
    return H4D_OK;
}

void set_lanes(h4d_system *s, int L) {
    s->a.lanes = L;
    s->a.lanes_log2 = L == 4 ? 2 : (L == 8 ? 3 : 4);
    s->a.step_blocks = s->a.slots / (kBlock / L);
}

int slot_blocks(const h4d_system *s) { return s->a.slots / kBlock; }

// Kept candidates of the cell-form list build held at once: as many as a
// quarter of the CU's 160 KB of LDS holds next to the centre atoms and the
// kernel's static arrays (four blocks per CU), and at least two passes of
// one candidate per thread.
int list_cand_cap(const h4d_system *s) {
    const int cap = s->a.cell_cap;
    const int fixed = (int)(2 * kWave * sizeof(uint4) + (size_t)cap * (sizeof(uint4) + sizeof(int)));
    constexpr int kStaticLds = 3072;  // the sub-cell range table (2,640 bytes) and slack
    return std::max(2 * kListWaves * kWave, (40 * 1024 - kStaticLds - fixed) / (int)sizeof(uint4));
}

// LDS of the cell-form list build: the staged candidates and their padding,
// the centre atoms and their running counts
size_t list_cells_lds(const h4d_system *s) {
    return (size_t)(list_cand_cap(s) + 2 * kWave) * sizeof(uint4) +
           (size_t)s->a.cell_cap * (sizeof(uint4) + sizeof(int));
}

// blocks per centre unit (sub-cell or cell) of the cell-form list build:
// the autotuner's choice, else enough blocks for two per CU (about 512 in
// all); at most 16 and at least two centre atoms of a full unit per
// wavefront
int list_split(const h4d_system *s) {
    const int unit_cap = s->a.cell_cap / s->list_units;
    const int most = std::max(1, std::min(16, unit_cap / (2 * kListWaves)));
    if (s->list_split > 0) return std::min(s->list_split, most);
    const int blocks = s->list_units * s->a.ncell_total;
    const int want = (512 + blocks - 1) / blocks;
    return std::max(1, std::min(want, most));
}

// list build; k and b as in list_wanted / buf_of
void launch_list(h4d_system *s, int k, int b, int cb, hipStream_t st) {
    KArgs &a = s->a;
    if (s->cells && list_cells_lds(s) <= 56 * 1024) {
        const int split = list_split(s), cand_cap = list_cand_cap(s), units = s->list_units;
        const dim3 grid(a.ncell_total * units * split), block(kListWaves * kWave);
        const size_t lds = list_cells_lds(s);
        if (a.G.water)
            hipLaunchKernelGGL(k_list_cells<true>, grid, block, lds, st, a, k, b, cb, split, cand_cap, units);
        else hipLaunchKernelGGL(k_list_cells<false>, grid, block, lds, st, a, k, b, cb, split, cand_cap, units);
    }
    else if (s->cells)
        hipLaunchKernelGGL(k_list_lanes, dim3(a.step_blocks), dim3(kBlock), 0, st, a, k, b, cb);
    else
        hipLaunchKernelGGL(k_list_allpairs, dim3(a.step_blocks), dim3(kBlock), 0, st, a, k, b, cb);
}

template <int PREC, int L, bool SP>
void launch_step_sp(h4d_system *s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int k, int b, int bin) {
    KArgs &a = s->a;
    const dim3 grid(a.step_blocks + s->nbox);
    if (PREC == 1 && nt_lists(s)) {
        if (e0) hipExtLaunchKernelGGL(k_step<PREC, L, SP, true>, grid, dim3(kBlock), 0, st, e0, e1, 0, a, k, b, bin, s->cl);
        else hipLaunchKernelGGL((k_step<PREC, L, SP, true>), grid, dim3(kBlock), 0, st, a, k, b, bin, s->cl);
    } else {
        if (e0) hipExtLaunchKernelGGL(k_step<PREC, L, SP, false>, grid, dim3(kBlock), 0, st, e0, e1, 0, a, k, b, bin, s->cl);
        else hipLaunchKernelGGL((k_step<PREC, L, SP, false>), grid, dim3(kBlock), 0, st, a, k, b, bin, s->cl);
    }
}

// species-specific w_max takes the kernels that give each flyer its own altitude
template <int PREC, int L>
void launch_step_l(h4d_system *s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int k, int b, int bin) {
    if (s->a.G.w_ratio != 1.0) launch_step_sp<PREC, L, true>(s, st, e0, e1, k, b, bin);
    else launch_step_sp<PREC, L, false>(s, st, e0, e1, k, b, bin);
}

template <int PREC>
void launch_step(h4d_system *s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int k, int b, int bin) {
    switch (s->a.lanes) {
        case 4: launch_step_l<PREC, 4>(s, st, e0, e1, k, b, bin); break;
        case 8: launch_step_l<PREC, 8>(s, st, e0, e1, k, b, bin); break;
        default: launch_step_l<PREC, 16>(s, st, e0, e1, k, b, bin); break;
    }
}

template <int PREC, bool SP>
void launch_forces_sp(h4d_system *s, double w) {
    KArgs &a = s->a;
    const dim3 grid(a.step_blocks);
    switch (a.lanes) {
        case 4: hipLaunchKernelGGL((k_forces<PREC, 4, SP>), grid, dim3(kBlock), 0, s->stream, a, w); break;
        case 8: hipLaunchKernelGGL((k_forces<PREC, 8, SP>), grid, dim3(kBlock), 0, s->stream, a, w); break;
        default: hipLaunchKernelGGL((k_forces<PREC, 16, SP>), grid, dim3(kBlock), 0, s->stream, a, w); break;
    }
}

template <int PREC>
void launch_forces(h4d_system *s, double w) {
    if (s->a.G.w_ratio != 1.0) launch_forces_sp<PREC, true>(s, w);
    else launch_forces_sp<PREC, false>(s, w);
}

// Sort the canonical atoms into cell order (working buffer 0), draw the
// momenta of each box's current trial index, and build the lists (cell
// buffer 0).
int sort_in(h4d_system *s, hipStream_t st) {
    KArgs &a = s->a;
    const int nc = a.ncell_total;
    hipLaunchKernelGGL(k_cell_clear, dim3(blocks_for(nc)), dim3(kBlock), 0, st, a, 0);
    hipLaunchKernelGGL(k_bin_canonical, dim3(slot_blocks(s)), dim3(kBlock), 0, st, a, 0);
    hipLaunchKernelGGL(k_cell_sort, dim3(nc), dim3(kWave), 3 * a.cell_cap * sizeof(int), st, a, 0);
    hipLaunchKernelGGL(k_cell_scan, dim3(s->nbox), dim3(1024), 0, st, a, 0);
    hipLaunchKernelGGL(k_gather_in, dim3(nc), dim3(kWave), 0, st, a, 0);
    if (a.G.water) hipLaunchKernelGGL(k_rattle_mb, dim3(blocks_for(a.G.n_mol * s->nbox)), dim3(kBlock), 0, st, a);
    launch_list(s, -1, 0, 0, st);
    s->cl = 0;
    HIPC(hipGetLastError());
    return H4D_OK;
}

// Rebuild before step k: the preceding step binned the atoms of every box
// still running into cell buffer cl ^ 1.
int rebuild_mid(h4d_system *s, int k, int b, hipStream_t st) {
    KArgs &a = s->a;
    const int cb = s->cl ^ 1;
    if (s->cells)
        hipLaunchKernelGGL(k_cell_sort, dim3(a.ncell_total), dim3(kWave), 3 * a.cell_cap * sizeof(int), st, a, cb);
    launch_list(s, k, b, cb, st);
    s->cl = cb;
    HIPC(hipGetLastError());
    return H4D_OK;
}

// End of the trajectories: lists of every box with a trajectory at its final
// state (no fast atoms), for the end energy.
int rebuild_final(h4d_system *s, hipStream_t st) {
    KArgs &a = s->a;
    const int cb = s->cl ^ 1;
    if (s->cells) {
        hipLaunchKernelGGL(k_cell_clear, dim3(blocks_for(a.ncell_total)), dim3(kBlock), 0, st, a, cb);
        hipLaunchKernelGGL(k_bin_working, dim3(slot_blocks(s)), dim3(kBlock), 0, st, a, cb);
        hipLaunchKernelGGL(k_cell_sort, dim3(a.ncell_total), dim3(kWave), 3 * a.cell_cap * sizeof(int), st, a, cb);
    }
    launch_list(s, -2, -1, cb, st);
    s->cl = cb;
    HIPC(hipGetLastError());
    return H4D_OK;
}

int read_ctl(h4d_system *s) {
    HIPC(hipMemcpyAsync(s->h_ctl, s->a.ctl, sizeof(Ctl) * s->nbox, hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int write_ctl(h4d_system *s) {
    HIPC(hipMemcpyAsync(s->a.ctl, s->h_ctl, sizeof(Ctl) * s->nbox, hipMemcpyHostToDevice, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int clear_errors(h4d_system *s) {
    int rc = read_ctl(s);
    if (rc) return rc;
    for (int b = 0; b < s->nbox; ++b) {
        Ctl *c = s->h_ctl + b;
        c->err = 0;
        c->retry = 0;
        c->max_nbr = 0;
        c->max_cell = 0;
    }
    return write_ctl(s);
}

// Grow the list storage after an overflow in any box.
int grow_lists(h4d_system *s, unsigned err, int max_nbr, int max_cell) {
    KArgs &a = s->a;
    if (err & kErrNbr) {
        int need = std::max(max_nbr, a.nbr_cap + kMaxLanes);
        need = (int)(need * 1.25) + kMaxLanes;
        need = round_up(need, kMaxLanes);
        s->release(a.nbr);
        a.nbr_cap = need;
        int rc = s->alloc(&a.nbr, nbr_elems(s));
        if (rc) return rc;
    }
    if (err & kErrCell) {
        int need = std::max(max_cell, a.cell_cap + 8);
        need = (int)(need * 1.25) + 8;
        s->release(a.cell_atoms[0]);
        s->release(a.cell_atoms[1]);
        a.cell_cap = need;
        int rc;
        if ((rc = s->alloc(&a.cell_atoms[0], (size_t)a.ncell_total * a.cell_cap))) return rc;
        if ((rc = s->alloc(&a.cell_atoms[1], (size_t)a.ncell_total * a.cell_cap))) return rc;
    }
    return H4D_OK;
}

// Candidates, features, logits and the multiple-try step of the learned
// proposal: phase 0 before an insertion's trajectory (working buffer 0, cell
// buffer 0), phase 1 after a deletion's (final buffer, last cell buffer).
void enqueue_learned(h4d_system *s, hipStream_t st, int phase, int b, int cb) {
    KArgs &a = s->a;
    const LearnArgs &l = s->la;
    const int rows = l.k * s->nbox;   // every box's candidates
    hipLaunchKernelGGL(k_cand_sites, dim3(blocks_for(rows)), dim3(kBlock), 0, st, a, l, phase);
    hipLaunchKernelGGL(k_site_features, dim3((int)((2 * (int64_t)rows * kWave + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, st, a, l, phase, b, cb);
    if (l.use_net) hipLaunchKernelGGL(k_mlp_infer_move, dim3((rows + 63) / 64), dim3(256), 0, st, a, l, phase);
    else hipLaunchKernelGGL(k_zero_logits, dim3(blocks_for(rows)), dim3(kBlock), 0, st, a, l, phase);
    hipLaunchKernelGGL(k_mtm_select, dim3(s->nbox), dim3(kMtmBlock), 0, st, a, l, phase);
}

// Enqueue every kernel of one round (each box's current trial) on st.  The
// round's shape is fixed by the rebuild interval and the largest N_f; the
// kernels read everything else from the control blocks.  With timing, HIP
// events bracket each step kernel.
int enqueue_round(h4d_system *s, int move, hipStream_t st, int nf, int M, bool timing) {
    KArgs &a = s->a;
    const int G1 = slot_blocks(s);
    int rc;
    hipLaunchKernelGGL(k_propose, dim3(s->nbox), dim3(kBlock), 0, st, a, move);
    if ((rc = sort_in(s, st))) return rc;
    if (s->la.k > 0 && move != kMoveMD) {   // learned insertion: score k candidates, move the ghosts, sort again
        enqueue_learned(s, st, 0, 0, 0);
        if ((rc = sort_in(s, st))) return rc;
    }
    hipLaunchKernelGGL(k_start_check, dim3(blocks_for(s->nbox)), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_energy, dim3(a.step_blocks), dim3(kBlock), 0, st, a, 0, -1, 0.0, 0);
    hipLaunchKernelGGL(k_energy_final, dim3(s->nbox), dim3(kBlock), 0, st, a, 0);
    int b = 0;
    for (int k = 0; k <= nf; ++k) {
        if (k > 0 && k % M == 0)
            if ((rc = rebuild_mid(s, k, b, st))) return rc;
        const int bin = s->cells && (k + 1) % M == 0 && k + 1 <= nf;
        hipEvent_t e0 = timing ? s->ev[2 * k] : nullptr, e1 = timing ? s->ev[2 * k + 1] : nullptr;
        if (s->p.precision == H4D_PREC_FP32) launch_step<1>(s, st, e0, e1, k, b, bin);
        else launch_step<0>(s, st, e0, e1, k, b, bin);
        if (a.G.water)
            hipLaunchKernelGGL(k_settle, dim3((a.G.n_mol * s->nbox + kSettleBlock - 1) / kSettleBlock),
                               dim3(kSettleBlock), 0, st, a, k, b, bin,
                               s->cl);
        b ^= 1;
    }
    if ((rc = rebuild_final(s, st))) return rc;
    hipLaunchKernelGGL(k_energy, dim3(a.step_blocks), dim3(kBlock), 0, st, a, 1, -1, 0.0, -1);
    hipLaunchKernelGGL(k_energy_final, dim3(s->nbox), dim3(kBlock), 0, st, a, 1);
    if (s->la.k > 0 && move != kMoveMD) enqueue_learned(s, st, 1, -1, s->cl);   // learned deletion: reverse weights
    if (a.G.bias_alpha > 0.0) hipLaunchKernelGGL(k_bias_end, dim3(s->nbox), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_metropolis, dim3(blocks_for(s->nbox)), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_commit, dim3(G1), dim3(kBlock), 0, st, a);
    if (a.G.water && move == kMoveMD)   // a rejected phase's reversed refresh, restricted
        hipLaunchKernelGGL(k_water_cvel, dim3(blocks_for(a.G.n_mol * s->nbox)), dim3(kBlock), 0, st, a, 1);
    hipLaunchKernelGGL(k_compact1, dim3(G1), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_compact2, dim3(G1), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_commit_ctl, dim3(blocks_for(s->nbox)), dim3(kBlock), 0, st, a);
    HIPC(hipGetLastError());
    return H4D_OK;
}

int launch_round(h4d_system *s, int move) {
    KArgs &a = s->a;
    hipStream_t st = s->stream;
    const int nf = move == kMoveMD ? a.md_steps : (s->p.n_steps_max > 0 ? s->p.n_steps_max : s->p.n_steps);
    if (move != kMoveMD) s->vel_canonical = false;
    const int M = std::max(1, s->trial_M);
    int rc;
    s->trial_rebuilds = nf / M + 1;
    if (s->timing && (int)s->ev.size() < 2 * (nf + 1)) {
        s->drop_graphs();
        while ((int)s->ev.size() < 2 * (nf + 1)) {
            hipEvent_t e;
            HIPC(hipEventCreate(&e));
            s->ev.push_back(e);
        }
    }
    bool launched = false;
    const int tm = s->timing ? 1 : 0;
    if (s->graphs_ok[tm]) {
        if (!s->cap_stream) HIPC(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
        const auto key = std::make_tuple(M, nf, move, tm, (a.lanes * 65536 + s->la.k) * 2 + (nt_lists(s) ? 1 : 0));
        auto it = s->graphs.find(key);
        if (it == s->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            bool ok = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            int erc = ok ? enqueue_round(s, move, s->cap_stream, nf, M, s->timing) : H4D_OK;
            ok = hipStreamEndCapture(s->cap_stream, &graph) == hipSuccess && ok && erc == H4D_OK;
            if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (ok) it = s->graphs.emplace(key, exec).first;
            else s->graphs_ok[tm] = false;   // capture unsupported: launch eagerly from now on
        }
        if (it != s->graphs.end()) {
            HIPC(hipGraphLaunch(it->second, st));
            launched = true;
        }
    }
    if (!launched && (rc = enqueue_round(s, move, st, nf, M, s->timing))) return rc;
    HIPC(hipMemcpyAsync(s->h_rec, a.rec, sizeof(TrialRec) * s->nbox, hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(s->h_ctl, a.ctl, sizeof(Ctl) * s->nbox, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (s->timing) {
        int nf_dev = 0;
        for (int b = 0; b < s->nbox; ++b) nf_dev = std::max(nf_dev, s->h_ctl[b].nf);
        nf_dev = std::min(nf_dev, nf);
        for (int k = 0; k <= nf_dev; ++k) {
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, s->ev[2 * k], s->ev[2 * k + 1]));
            s->step_ms += ms;
            s->step_launches += 1;
        }
        // a box's trajectory runs in launches k = 0..N_f of the round; its
        // blocks of the later ones return at once
        for (int b = 0; b < s->nbox; ++b) {
            const TrialRec &r = s->h_rec[b];
            if (r.flags & kFlagIdle) continue;
            s->atom_launches += (double)r.n_atoms * (double)(std::min(r.n_steps, nf_dev) + 1);
        }
    }
    return H4D_OK;
}

// After a round: boxes that must recompute their trial (list overflow, fast
// list full, atom capacity) get larger buffers or a shorter rebuild interval.
// Returns the number of boxes to recompute.
int handle_retries(h4d_system *s, int &rc) {
    rc = H4D_OK;
    unsigned err = 0;
    int max_nbr = 0, max_cell = 0, n = 0;
    for (int b = 0; b < s->nbox; ++b) {
        const Ctl *c = s->h_ctl + b;
        if (!c->retry) continue;
        ++n;
        err |= c->err;
        max_nbr = std::max(max_nbr, c->max_nbr);
        max_cell = std::max(max_cell, c->max_cell);
    }
    if (!n) return 0;
    if (err & kErrCap) { rc = fail(H4D_ECAPACITY, "atom capacity exhausted"); return n; }
    if ((rc = grow_lists(s, err, max_nbr, max_cell))) return n;
    // more fast atoms than the fast list holds: recompute with a shorter
    // rebuild interval, and shorten the base interval
    if (err & (kErrSkin | kErrFast)) {
        s->trial_M = std::max(1, s->trial_M / 2);
        if (s->p.rebuild_every == 0) s->rebuild_every = std::max(1, (s->rebuild_every * 3) / 4);
        s->clean_trials = 0;
    }
    rc = clear_errors(s);
    s->retries += n;
    s->retries_total += n;
    return n;
}

// Book-keeping of a finished trial of box b.
void account(h4d_system *s, int b, const h4d_trial &r) {
    const Ctl *c = s->h_ctl + b;
    h4d_system::Stats &st = s->stats[b];
    s->n_host[b] = c->n;
    s->nsalt_host[b] = c->nsalt;
    st.n_trials += 1;
    if (r.flags & kFlagNonfinite) s->nonfinite += 1;
    if (r.move > 0) { st.n_ins += 1; st.n_ins_acc += r.accepted; }
    else { st.n_del += 1; st.n_del_acc += r.accepted; }
    st.N_sum += (double)c->nsalt;
    st.N2_sum += (double)c->nsalt * (double)c->nsalt;
}

// automatic rebuild interval: lengthen it after a run of rounds whose fast
// lists stayed short (a few percent of their capacity)
void adapt_interval(h4d_system *s) {
    if (s->p.rebuild_every != 0 || s->interval_tuned) return;
    int mf = 0;
    for (int b = 0; b < s->nbox; ++b) mf = std::max(mf, s->h_ctl[b].max_fast);
    if (mf <= kFastCap / 16) {
        if (++s->clean_trials >= 20) { s->rebuild_every += 1; s->clean_trials = 0; }
    } else {
        s->clean_trials = 0;
    }
}

int run_one(h4d_system *s, int move, h4d_trial *out) {
    bool retried = false;
    s->trial_M = std::max(1, s->rebuild_every);
    for (int attempt = 0; attempt < 16; ++attempt) {
        int rc = launch_round(s, move);
        if (rc) return rc;
        if (handle_retries(s, rc)) {
            if (rc) return rc;
            retried = true;
            continue;
        }
        h4d_trial r;
        std::memcpy(&r, s->h_rec, sizeof(r));
        if (retried) r.flags |= H4D_FLAG_RETRIED;
        r.n_rebuilds = s->trial_rebuilds;
        if (out) *out = r;
        account(s, 0, r);
        if (!retried) adapt_interval(s);
        return H4D_OK;
    }
    return fail(H4D_EHIP, "trial could not be completed after resizing the lists");
}

int set_quota(h4d_system *s, long long count) {
    hipLaunchKernelGGL(k_set_quota, dim3(blocks_for(s->nbox)), dim3(kBlock), 0, s->stream, s->a, count);
    HIPC(hipGetLastError());
    return read_ctl(s);
}

int run_batch(h4d_system *s, int T, int move, h4d_trial *out, int active = -1) {
    int rc = set_quota(s, T);
    if (rc) return rc;
    if (active >= 0 && active < s->nbox) {   // boxes from `active` on sit this batch out
        for (int b = active; b < s->nbox; ++b) s->h_ctl[b].trial_end = s->h_ctl[b].trial;
        if ((rc = write_ctl(s))) return rc;
    }
    std::vector<long long> first(s->nbox);
    std::vector<char> retried(s->nbox, 0);
    for (int b = 0; b < s->nbox; ++b) first[b] = s->h_ctl[b].trial;
    const int max_rounds = T + 64;
    int rounds = 0;
    bool any_retry = false;
    for (;;) {
        bool busy = false;
        for (int b = 0; b < s->nbox; ++b) busy |= s->h_ctl[b].trial < s->h_ctl[b].trial_end;
        if (!busy) break;
        if (++rounds > max_rounds) {
            (void)set_quota(s, -1);
            return fail(H4D_EHIP, "batch could not be completed after resizing the lists");
        }
        // the base interval, unless the last round had to recompute a trial
        // (then the interval handle_retries shortened stays for this round)
        if (!any_retry) s->trial_M = std::max(1, s->rebuild_every);
        if ((rc = launch_round(s, move))) return rc;
        any_retry = false;
        for (int b = 0; b < s->nbox; ++b) {
            const Ctl *c = s->h_ctl + b;
            const TrialRec &tr = s->h_rec[b];
            if (tr.flags & kFlagIdle) continue;
            if (c->retry) { retried[b] = 1; any_retry = true; continue; }
            h4d_trial r;
            std::memcpy(&r, &tr, sizeof(r));
            if (retried[b]) r.flags |= H4D_FLAG_RETRIED;
            retried[b] = 0;
            r.n_rebuilds = s->trial_rebuilds;
            const long long q = r.trial - first[b];
            if (out && q >= 0 && q < T) out[(size_t)b * T + q] = r;
            account(s, b, r);
        }
        if (any_retry) {
            handle_retries(s, rc);
            if (rc) { (void)set_quota(s, -1); return rc; }
            if ((rc = read_ctl(s))) return rc;
        } else {
            adapt_interval(s);
        }
    }
    return set_quota(s, -1);
}

// Carried momenta on speculative replicas: replica b runs trial t0 + b, which
// follows b rejected trials of the chain.  Each of those reversed the
// momenta by the product of its two reversal signs (a trial with a pair to
// delete, or any insertion, moves), so the replica starts from the chain's
// momenta times those b products.
__global__ __launch_bounds__(kBlock) void k_spec_momenta(KArgs a, long long t0) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.slots) return;
    const int bi = box_of_slot(a, i);
    const Box &B = a.box[bi];
    if (bi == 0 || i - B.a0 >= a.ctl[bi].n) return;
    double sgn = 1.0;
    for (int j = 0; j < bi; ++j) sgn *= reversal_sign(a, B, t0 + j, 0) * reversal_sign(a, B, t0 + j, 1);
    const double4 v = a.cvel[i];
    a.cvel[i] = make_double4(sgn * v.x, sgn * v.y, sgn * v.z, v.w);
}

// One equilibrium phase of every box (its records in out[b]); a box whose
// phase overflowed a list repeats it after the resize while the others idle.
int run_md(h4d_system *s, int n_steps, h4d_trial *out) {
    KArgs &a = s->a;
    if (a.md_steps != n_steps) {
        a.md_steps = n_steps;
        s->drop_graphs();     // the graphs captured the step count
    }
    int rc;
    if (s->speculative) {
        // the replicas hold one chain: the phase runs on replica 0 alone and
        // the others take its state afterwards
        if ((rc = read_ctl(s))) return rc;
        for (int b = 0; b < s->nbox; ++b) s->h_ctl[b].md_end = s->h_ctl[b].md + (b == 0 ? 1 : 0);
        if ((rc = write_ctl(s))) return rc;
    } else {
        hipLaunchKernelGGL(k_set_md_quota, dim3(blocks_for(s->nbox)), dim3(kBlock), 0, s->stream, a, 1LL);
        HIPC(hipGetLastError());
        if ((rc = read_ctl(s))) return rc;
    }
    s->trial_M = std::max(1, s->rebuild_every);
    for (int round = 0; round < 64; ++round) {
        bool busy = false;
        for (int b = 0; b < s->nbox; ++b) busy |= s->h_ctl[b].md < s->h_ctl[b].md_end;
        if (!busy) {
            if (s->speculative && s->nbox > 1) {
                hipLaunchKernelGGL(k_broadcast_box, dim3(slot_blocks(s)), dim3(kBlock), 0, s->stream, a, 0);
                HIPC(hipGetLastError());
                if ((rc = read_ctl(s))) return rc;
                for (int b = 1; b < s->nbox; ++b) {
                    s->n_host[b] = s->n_host[0];
                    s->nsalt_host[b] = s->nsalt_host[0];
                    if (out) out[b] = out[0];
                }
            }
            s->vel_canonical = true;
            return H4D_OK;
        }
        if ((rc = launch_round(s, kMoveMD))) return rc;
        bool any_retry = false;
        for (int b = 0; b < s->nbox; ++b) {
            const TrialRec &tr = s->h_rec[b];
            if (tr.flags & kFlagIdle) continue;
            if (s->h_ctl[b].retry) { any_retry = true; continue; }
            h4d_trial r;
            std::memcpy(&r, &tr, sizeof(r));
            r.n_rebuilds = s->trial_rebuilds;
            if (out) out[b] = r;
        }
        if (any_retry) {
            handle_retries(s, rc);
            if (rc) return rc;
            if ((rc = read_ctl(s))) return rc;
        }
    }
    return fail(H4D_EHIP, "equilibrium phase could not be completed after resizing the lists");
}

int create(const h4d_params *params, int nbox, const double *edges, const int32_t *n_atoms, const int32_t *n_salt,
           int32_t n_mol, const double *pos, const int32_t *type, const int32_t *mol, const int64_t *tag,
           void *hip_stream, h4d_system **out, bool speculative = false) {
    g_err.clear();
    if (!params || !out || nbox < 1 || !edges || !n_atoms || !n_salt) return fail(H4D_EINVAL, "null argument");
    *out = nullptr;
    int rc = check_params(*params);
    if (rc) return rc;
    long long total = 0;
    for (int b = 0; b < nbox; ++b) {
        if (n_atoms[b] < 0 || n_salt[b] < 0) return fail(H4D_EINVAL, "negative size");
        total += n_atoms[b];
    }
    if (total > 0 && (!pos || !type || !tag)) return fail(H4D_EINVAL, "null configuration array");
    if (params->water && nbox != 1 && !speculative)
        return fail(H4D_EINVAL, "rigid water needs a single box (or speculative replicas)");
    const double rc_max = std::max(params->rc_lj, params->rc_coul);
    for (int q = 0; q < 3 * nbox; ++q)
        if (!(edges[q] >= 2.0 * rc_max)) return fail(H4D_EINVAL, "every box edge must be at least twice the largest cutoff");
    int ndev = 0;
    const hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1)
        return fail(H4D_ENODEV, std::string("no HIP device (hipGetDeviceCount: ") + hipGetErrorString(de) +
                                    ", count " + std::to_string(ndev) + ")");
    // validate the configuration, box by box
    long long off = 0;
    for (int b = 0; b < nbox; ++b) {
        int ncat = 0, nan_ = 0;
        for (int q = 0; q < n_atoms[b]; ++q) {
            const long long i = off + q;
            if (type[i] < 0 || type[i] >= params->n_types) return fail(H4D_EINVAL, "atom type out of range");
            ncat += type[i] == params->cation_type;
            nan_ += type[i] == params->anion_type;
            if (q > 0 && tag[i] <= tag[i - 1]) return fail(H4D_EINVAL, "tags must ascend in array order within a box");
            for (int d = 0; d < 3; ++d)
                if (!(pos[3 * i + d] >= 0.0 && pos[3 * i + d] < edges[3 * b + d]))
                    return fail(H4D_EINVAL, "positions must lie in [0, L)");
        }
        if (ncat != n_salt[b] || nan_ != n_salt[b])
            return fail(H4D_EINVAL, "n_salt must equal the cation and anion counts of each box");
        off += n_atoms[b];
    }
    const int n0 = n_atoms[0];
    if (params->water) {
        if (n_mol < 1 || 3 * n_mol > n0 || !mol) return fail(H4D_EINVAL, "water = 1 needs n_mol >= 1 waters first");
        for (int m = 0; m < n_mol; ++m)
            for (int q = 0; q < 3; ++q) {
                const int i = 3 * m + q;
                if (mol[i] != m || type[i] != type[q]) return fail(H4D_EINVAL, "waters must be atoms 3m, 3m+1, 3m+2 (O, H, H) of molecule m");
            }
        if (type[1] != type[2] || type[0] == type[1]) return fail(H4D_EINVAL, "water atoms must be O, H, H");
        for (int i = 3 * n_mol; i < n0; ++i)
            if (mol[i] >= 0) return fail(H4D_EINVAL, "only the waters may carry molecule ids");
    } else if (mol) {
        for (long long i = 0; i < total; ++i)
            if (mol[i] >= 0) return fail(H4D_EINVAL, "molecule ids need water = 1");
    }

    auto *s = new h4d_system();
    s->p = *params;
    s->nbox = nbox;
    if (const char *e = std::getenv("H4D_NO_GRAPHS")) {
        if (e[0] == '1') s->graphs_ok[0] = false;   // launch every kernel eagerly
    }
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->speculative = speculative;
    s->n_mol = n_mol;
    s->n_host.assign(n_atoms, n_atoms + nbox);
    s->nsalt_host.assign(n_salt, n_salt + nbox);
    s->stats.assign(nbox, h4d_system::Stats{});
    setup_geo(s);
    if ((rc = setup_boxes(s, edges, n_atoms))) { delete s; return rc; }
    if ((rc = setup_bias(s, params->bias_xb, params->bias_alpha))) { delete s; return rc; }
    if (params->water) {
        Geo &G = s->a.G;
        G.n_mol = n_mol;
        G.m_o = params->mass[type[0]];
        G.m_h = params->mass[type[1]];
        G.rc_w = 0.5 * params->d_hh;
        const double h = std::sqrt(params->d_oh * params->d_oh - G.rc_w * G.rc_w);
        G.ra = 2.0 * G.m_h * h / (G.m_o + 2.0 * G.m_h);
        G.rb = h - G.ra;
    }
    {
        int L = params->lanes_per_atom;
        int nmax = 0;
        for (int b = 0; b < nbox; ++b) nmax = std::max(nmax, n_atoms[b]);
        if (L == 0) L = (long long)total <= 16384 ? 16 : (total <= 65536 && nmax <= 65536 ? 8 : 4);
        set_lanes(s, L);
    }
    initial_capacities(s, n_atoms);
    KArgs &a = s->a;
    a.seed = params->seed;
    a.n_steps = params->n_steps;
    a.n_steps_min = params->n_steps_min;
    a.n_steps_max = params->n_steps_max;
    a.cation_type = params->cation_type;
    a.anion_type = params->anion_type;
    s->partial_blocks = a.slots / (kBlock / kMaxLanes);   // every energy grid fits
    const size_t C = (size_t)a.slots;
    PairCoef *coef_d = nullptr;
    double *mass_d = nullptr;
    Box *box_d = nullptr;
    int *slot_box_d = nullptr, *cell_box_d = nullptr;
    if ((rc = s->alloc(&a.cpos, C)) || (rc = s->alloc(&a.cvel, C)) || (rc = s->alloc(&a.tvel, C)) ||
        (rc = s->alloc(&a.ctag, C)) || (rc = s->alloc(&a.ctype, C)) ||
        (rc = s->alloc(&a.cmol, C)) || (rc = s->alloc(&a.pos[0], C + 1)) || (rc = s->alloc(&a.pos[1], C + 1)) ||
        (rc = s->alloc(&a.fx[0], C + 1)) || (rc = s->alloc(&a.fx[1], C + 1)) || (rc = s->alloc(&a.vel[0], C)) ||
        (rc = s->alloc(&a.vel[1], C)) || (rc = s->alloc(&a.perm, C)) || (rc = s->alloc(&a.wmol, C)) ||
        (rc = s->alloc(&a.posb, C)) || (rc = s->alloc(&a.force, C)) || (rc = s->alloc(&a.tpos, C)) ||
        (rc = s->alloc(&a.ttag, C)) || (rc = s->alloc(&a.ttype, C)) || (rc = s->alloc(&a.tmol, C)) ||
        (rc = s->alloc(&a.nnbr, C)) || (rc = s->alloc(&a.partial, (size_t)s->partial_blocks * 5)) ||
        (rc = s->alloc(&a.ctl, (size_t)nbox)) || (rc = s->alloc(&a.rec, (size_t)nbox)) ||
        (rc = s->alloc(&a.molw, n_mol > 0 ? C : 1)) || (rc = s->alloc(&a.fw, C)) ||
        (rc = s->alloc(&coef_d, (size_t)kMaxTypes * kMaxTypes)) || (rc = s->alloc(&mass_d, kMaxTypes)) ||
        (rc = s->alloc(&box_d, (size_t)nbox)) || (rc = s->alloc(&slot_box_d, C / kBlock)) ||
        (rc = s->alloc(&cell_box_d, (size_t)a.ncell_total)) || (rc = alloc_lists(s))) {
        delete s;
        return rc;
    }
    a.coef = coef_d;
    a.mass = mass_d;
    a.box = box_d;
    a.slot_box = slot_box_d;
    a.cell_box = cell_box_d;
    if (hipHostMalloc((void **)&s->h_rec, sizeof(TrialRec) * nbox) != hipSuccess ||
        hipHostMalloc((void **)&s->h_ctl, sizeof(Ctl) * nbox) != hipSuccess) {
        delete s;
        return fail(H4D_ENOMEM, "pinned host allocation failed");
    }
    // upload: each box's atoms at its slots, rest of the slots zero
    std::vector<double4> hp(C, make_double4(0.0, 0.0, 0.0, 0.0));
    std::vector<int> ht(C, 0), hm(C, -1);
    std::vector<long long> hg(C, 0);
    std::vector<int> sb(C / kBlock), cbx(a.ncell_total);
    std::memset(s->h_ctl, 0, sizeof(Ctl) * nbox);
    off = 0;
    for (int b = 0; b < nbox; ++b) {
        const Box &B = s->box_h[b];
        for (int q = 0; q < n_atoms[b]; ++q) {
            const long long i = off + q;
            const int w = B.a0 + q;
            long long meta = type[i];
            double wbits;
            std::memcpy(&wbits, &meta, sizeof(wbits));
            hp[w] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], wbits);
            ht[w] = type[i];
            hg[w] = tag[i];
            if (mol) hm[w] = mol[i];
        }
        for (int q = B.a0 / kBlock; q < (B.a0 + B.cap) / kBlock; ++q) sb[q] = b;
        for (int q = B.c0; q < B.c0 + B.nc; ++q) cbx[q] = b;
        Ctl &c = s->h_ctl[b];
        c.n = n_atoms[b];
        c.n_all = n_atoms[b];
        c.nsalt = n_salt[b];
        c.next_tag = n_atoms[b] ? tag[off + n_atoms[b] - 1] + 1 : 0;
        c.trial = 0;
        c.trial_end = 0x7fffffffffffffffLL;
        c.ic = c.ia = -1;
        off += n_atoms[b];
    }
    double mass_h[kMaxTypes] = {0};
    for (int t = 0; t < params->n_types; ++t) mass_h[t] = params->mass[t];
#define UPLOAD(dst, src, bytes)                                                                        \
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {                           \
        delete s;                                                                                      \
        return fail(H4D_EHIP, "upload failed");                                                       \
    }
    UPLOAD(a.cpos, hp.data(), sizeof(double4) * C);
    UPLOAD(a.ctype, ht.data(), sizeof(int) * C);
    UPLOAD(a.cmol, hm.data(), sizeof(int) * C);
    UPLOAD(a.ctag, hg.data(), sizeof(long long) * C);
    UPLOAD(a.ctl, s->h_ctl, sizeof(Ctl) * nbox);
    UPLOAD(coef_d, s->coef_h, sizeof(s->coef_h));
    UPLOAD(mass_d, mass_h, sizeof(mass_h));
    UPLOAD(box_d, s->box_h.data(), sizeof(Box) * nbox);
    UPLOAD(slot_box_d, sb.data(), sizeof(int) * sb.size());
    UPLOAD(cell_box_d, cbx.data(), sizeof(int) * cbx.size());
    {   // the null record past the last slot: the pair pass pads the lists with
        // it (its fast flag gives exactly zero force); the list build's
        // padding entries carry its slot
        const uint4 null_rec = make_uint4(0u, 0u, 0u, (unsigned)kFastBit);
        UPLOAD(a.fx[0] + C, &null_rec, sizeof(uint4));
        UPLOAD(a.fx[1] + C, &null_rec, sizeof(uint4));
        long long meta = kFastBit;
        double wbits;
        std::memcpy(&wbits, &meta, sizeof(wbits));
        const double4 null_pos = make_double4(0.0, 0.0, 0.0, wbits);
        UPLOAD(a.pos[0] + C, &null_pos, sizeof(double4));
        UPLOAD(a.pos[1] + C, &null_pos, sizeof(double4));
    }
#undef UPLOAD
    // rebuild interval: the fastest atoms (5 standard deviations) cover half
    // the skin; adapted on overflow
    double m_min = params->mass[0];
    for (int t = 1; t < params->n_types; ++t) m_min = std::min(m_min, params->mass[t]);
    const double vmax = 5.0 * std::sqrt(params->accel * params->kT / m_min);
    s->rebuild_every = params->rebuild_every > 0
                           ? params->rebuild_every
                           : std::max(1, (int)std::floor(0.5 * params->skin / (vmax * params->dt)));
    {   // the state's own momenta (carried momenta, equilibrium phases); rigid
        // waters' restricted to the constraint surface
        hipLaunchKernelGGL(k_init_velocities, dim3(slot_blocks(s)), dim3(kBlock), 0, s->stream, s->a);
        if (params->water)
            hipLaunchKernelGGL(k_water_cvel, dim3(blocks_for(s->a.G.n_mol * s->nbox)), dim3(kBlock), 0, s->stream,
                               s->a, 0);
        if (hipGetLastError() != hipSuccess) { delete s; return fail(H4D_EHIP, "velocity set-up failed"); }
        s->vel_canonical = true;
    }
    if ((rc = h4d_build_neighbors(s))) { delete s; return rc; }
    *out = s;
    return H4D_OK;
}

// FP64 energies of every box's working buffer-0 state (after sort_in); the
// results of box b are left in h_ctl[b].
int energies(h4d_system *s) {
    KArgs &a = s->a;
    hipLaunchKernelGGL(k_energy, dim3(a.step_blocks), dim3(kBlock), 0, s->stream, a, 2, 0, 0.0, 0);
    hipLaunchKernelGGL(k_energy_final, dim3(s->nbox), dim3(kBlock), 0, s->stream, a, 2);
    HIPC(hipGetLastError());
    return read_ctl(s);
}

int box_state(h4d_system *s, int box, int32_t cap, int32_t *n, int32_t *n_salt, double *pos, double *vel,
              int32_t *type, int32_t *mol, int64_t *tag) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (box < 0 || box >= s->nbox) return fail(H4D_EINVAL, "box index out of range");
    int rc = read_ctl(s);
    if (rc) return rc;
    const Ctl &c = s->h_ctl[box];
    const Box &B = s->box_h[box];
    const int nn = c.n;
    if (n) *n = nn;
    if (n_salt) *n_salt = c.nsalt;
    if ((pos || vel || type || mol || tag) && cap < nn) return fail(H4D_EINVAL, "cap smaller than the atom count");
    std::vector<double4> buf(std::max(1, nn));
    if (pos && nn) {
        HIPC(hipMemcpy(buf.data(), s->a.cpos + B.a0, sizeof(double4) * nn, hipMemcpyDeviceToHost));
        for (int i = 0; i < nn; ++i) { pos[3 * i] = buf[i].x; pos[3 * i + 1] = buf[i].y; pos[3 * i + 2] = buf[i].z; }
    }
    if (vel && nn && (s->p.momenta || s->vel_canonical)) {
        // the state's own momenta (carried momenta, or after an equilibrium phase)
        HIPC(hipMemcpy(buf.data(), s->a.cvel + B.a0, sizeof(double4) * nn, hipMemcpyDeviceToHost));
        for (int i = 0; i < nn; ++i) { vel[3 * i] = buf[i].x; vel[3 * i + 1] = buf[i].y; vel[3 * i + 2] = buf[i].z; }
    } else if (vel && nn) {
        // velocities are those of the last trajectory's end, in canonical order
        std::vector<int> perm(nn);
        HIPC(hipMemcpy(perm.data(), s->a.perm + B.a0, sizeof(int) * nn, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(buf.data(), s->a.vel[(c.nf + 1) & 1] + B.a0, sizeof(double4) * nn, hipMemcpyDeviceToHost));
        for (int w = 0; w < nn; ++w) {
            const int i = perm[w] - B.a0;
            if (i < 0 || i >= nn) continue;
            vel[3 * i] = buf[w].x; vel[3 * i + 1] = buf[w].y; vel[3 * i + 2] = buf[w].z;
        }
    }
    if (type && nn) HIPC(hipMemcpy(type, s->a.ctype + B.a0, sizeof(int) * nn, hipMemcpyDeviceToHost));
    if (mol && nn) HIPC(hipMemcpy(mol, s->a.cmol + B.a0, sizeof(int) * nn, hipMemcpyDeviceToHost));
    if (tag && nn) HIPC(hipMemcpy(tag, s->a.ctag + B.a0, sizeof(long long) * nn, hipMemcpyDeviceToHost));
    return H4D_OK;
}

int box_observables(h4d_system *s, int box, h4d_observables *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    if (box < 0 || box >= s->nbox) return fail(H4D_EINVAL, "box index out of range");
    int rc = h4d_build_neighbors(s);
    if (rc) return rc;
    if ((rc = energies(s))) return rc;
    std::memset(out, 0, sizeof(*out));
    const Ctl *c = s->h_ctl + box;
    const h4d_system::Stats &st = s->stats[box];
    out->n_atoms = c->n;
    out->n_salt = c->nsalt;
    out->n_trials = st.n_trials;
    out->n_ins = st.n_ins;
    out->n_ins_acc = st.n_ins_acc;
    out->n_del = st.n_del;
    out->n_del_acc = st.n_del_acc;
    out->U = c->Ulj + c->Uc;
    out->U_lj = c->Ulj;
    out->U_coul = c->Uc;
    out->virial = c->vir;
    out->pressure_virial = ((double)c->n * s->p.kT + c->vir / 3.0) / s->box_h[box].volume;
    if (st.n_trials > 0) {
        out->N_mean = st.N_sum / (double)st.n_trials;
        out->N2_mean = st.N2_sum / (double)st.n_trials;
        out->chi = out->N_mean > 0.0 ? (out->N2_mean - out->N_mean * out->N_mean) / out->N_mean : 0.0;
    }
    return H4D_OK;
}

}  // namespace

extern "C" {

const char *h4d_last_error(void) { return g_err.c_str(); }

int32_t h4d_init_system(const h4d_params *params, int32_t n_atoms, int32_t n_salt, int32_t n_mol,
                        const double *pos, const int32_t *type, const int32_t *mol, const int64_t *tag,
                        void *hip_stream, h4d_system **out) {
    if (!params) return fail(H4D_EINVAL, "null argument");
    return create(params, 1, params->box, &n_atoms, &n_salt, n_mol, pos, type, mol, tag, hip_stream, out);
}

int32_t h4d_init_batch(const h4d_params *params, int32_t n_boxes, const double *box_edges,
                       const int32_t *n_atoms, const int32_t *n_salt, const double *pos, const int32_t *type,
                       const int64_t *tag, void *hip_stream, h4d_system **out) {
    if (n_boxes < 1) return fail(H4D_EINVAL, "n_boxes must be >= 1");
    return create(params, n_boxes, box_edges, n_atoms, n_salt, 0, pos, type, nullptr, tag, hip_stream, out);
}

int32_t h4d_num_boxes(const h4d_system *s) { return s ? s->nbox : 0; }

int32_t h4d_init_speculative(const h4d_params *params, int32_t replicas, int32_t n_atoms, int32_t n_salt,
                             int32_t n_mol, const double *pos, const int32_t *type, const int32_t *mol,
                             const int64_t *tag, void *hip_stream, h4d_system **out) {
    if (!params || !out) return fail(H4D_EINVAL, "null argument");
    if (replicas < 1 || replicas > 64) return fail(H4D_EINVAL, "replicas must be in 1..64");
    if (n_atoms < 0 || (n_atoms > 0 && (!pos || !type || !tag))) return fail(H4D_EINVAL, "null configuration array");
    const size_t n = (size_t)n_atoms, K = (size_t)replicas;
    std::vector<double> edges(3 * K), p(3 * n * K);
    std::vector<int32_t> na(K, n_atoms), ns(K, n_salt), ty(n * K), mo(mol ? n * K : 0);
    std::vector<int64_t> tg(n * K);
    for (size_t r = 0; r < K; ++r) {
        for (int d = 0; d < 3; ++d) edges[3 * r + d] = params->box[d];
        std::copy(pos, pos + 3 * n, p.begin() + 3 * n * r);
        std::copy(type, type + n, ty.begin() + n * r);
        std::copy(tag, tag + n, tg.begin() + n * r);
        if (mol) std::copy(mol, mol + n, mo.begin() + n * r);
    }
    return create(params, replicas, edges.data(), na.data(), ns.data(), n_mol, p.data(), ty.data(),
                  mol ? mo.data() : nullptr, tg.data(), hip_stream, out, true);
}

int32_t h4d_run_md(h4d_system *s, int32_t n_steps, h4d_trial *out) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (n_steps < 1) return fail(H4D_EINVAL, "n_steps must be at least 1");
    return run_md(s, n_steps, out);
}

int32_t h4d_run_speculative(h4d_system *s, int32_t n_trials, int32_t move, h4d_trial *out, int32_t *rounds_out) {
    if (!s || n_trials < 0 || (n_trials > 0 && !out)) return fail(H4D_EINVAL, "null handle or output");
    if (!s->speculative) return fail(H4D_EINVAL, "not a speculative handle (h4d_init_speculative)");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    const int K = s->nbox;
    std::vector<h4d_trial> recs(K);
    int rc = read_ctl(s);
    if (rc) return rc;
    long long t0 = s->h_ctl[0].trial;
    int done = 0, rounds = 0;
    const bool carry = s->p.momenta != 0;
    while (done < n_trials) {
        // With carried momenta and no salt, a drawn deletion makes no move
        // and no reversal, so the replicas' start momenta are not known in
        // advance: such a round runs the first replica alone.
        const int Ka = (carry && s->nsalt_host[0] == 0) ? 1 : K;
        // replica b runs trial t0 + b of the chain from the chain's state
        for (int b = 0; b < K; ++b) s->h_ctl[b].trial = t0 + b;
        if ((rc = write_ctl(s))) return rc;
        if (carry && Ka > 1) {
            hipLaunchKernelGGL(k_spec_momenta, dim3(slot_blocks(s)), dim3(kBlock), 0, s->stream, s->a, t0);
            HIPC(hipGetLastError());
        }
        if ((rc = run_batch(s, 1, move, recs.data(), Ka))) return rc;
        ++rounds;
        // the chain's trials: up to and including the first accepted one
        bool any = false;
        for (int b = 0; b < Ka; ++b) any |= recs[b].accepted != 0;
        int m = 0;
        while (m < Ka && done + m < n_trials) {
            const h4d_trial &r = recs[m];
            out[done + m] = r;
            h4d_system::Stats &st = s->chain;
            st.n_trials += 1;
            if (r.move > 0) { st.n_ins += 1; st.n_ins_acc += r.accepted; }
            else { st.n_del += 1; st.n_del_acc += r.accepted; }
            st.N_sum += (double)r.n_salt_after;
            st.N2_sum += (double)r.n_salt_after * (double)r.n_salt_after;
            ++m;
            if (r.accepted) break;
        }
        if (any || (carry && K > 1)) {   // every replica takes the state after the chain's last trial
            // (with carried momenta also after rejections: the momenta of
            // the chain's last trial's replica carry all their reversals)
            const int src = m - 1;
            hipLaunchKernelGGL(k_broadcast_box, dim3(slot_blocks(s)), dim3(kBlock), 0, s->stream, s->a, src);
            HIPC(hipGetLastError());
            if ((rc = read_ctl(s))) return rc;
            for (int b = 0; b < K; ++b) { s->n_host[b] = s->n_host[src]; s->nsalt_host[b] = s->nsalt_host[src]; }
        }
        done += m;
        t0 += m;
    }
    if ((rc = read_ctl(s))) return rc;
    for (int b = 0; b < K; ++b) { s->h_ctl[b].trial = t0; s->stats[b] = s->chain; }
    if ((rc = write_ctl(s))) return rc;
    if (rounds_out) *rounds_out = rounds;
    return H4D_OK;
}

int32_t h4d_build_neighbors(h4d_system *s) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    for (int attempt = 0; attempt < 8; ++attempt) {
        int rc = sort_in(s, s->stream);
        if (rc) return rc;
        if ((rc = read_ctl(s))) return rc;
        unsigned err = 0;
        int max_nbr = 0, max_cell = 0;
        for (int b = 0; b < s->nbox; ++b) {
            err |= s->h_ctl[b].err;
            max_nbr = std::max(max_nbr, s->h_ctl[b].max_nbr);
            max_cell = std::max(max_cell, s->h_ctl[b].max_cell);
        }
        if (!(err & (kErrNbr | kErrCell))) return H4D_OK;
        if ((rc = grow_lists(s, err, max_nbr, max_cell))) return rc;
        if ((rc = clear_errors(s))) return rc;
    }
    return fail(H4D_ECAPACITY, "neighbour lists could not be sized");
}

int32_t h4d_run_nemd_trial(h4d_system *s, int32_t move, h4d_trial *out) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (s->nbox != 1) return fail(H4D_EINVAL, "a batch of boxes runs with h4d_run_batch");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    return run_one(s, move, out);
}

int32_t h4d_run_trials(h4d_system *s, int32_t n, int32_t move, h4d_trial *out) {
    if (!s || n < 0) return fail(H4D_EINVAL, "null handle or negative count");
    if (s->nbox != 1) return fail(H4D_EINVAL, "a batch of boxes runs with h4d_run_batch");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    for (int q = 0; q < n; ++q) {
        int rc = run_one(s, move, out ? out + q : nullptr);
        if (rc) return rc;
    }
    return H4D_OK;
}

int32_t h4d_run_batch(h4d_system *s, int32_t trials_per_box, int32_t move, h4d_trial *out) {
    if (!s || trials_per_box < 0) return fail(H4D_EINVAL, "null handle or negative count");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    if (trials_per_box == 0) return H4D_OK;
    return run_batch(s, trials_per_box, move, out);
}

int32_t h4d_set_beta_mu(h4d_system *s, double beta_mu) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (!std::isfinite(beta_mu)) return fail(H4D_EINVAL, "beta_mu must be finite");
    s->p.beta_mu = beta_mu;
    s->a.G.beta_mu = beta_mu;
    s->drop_graphs();       // the captured launches hold the old value
    return H4D_OK;
}

int32_t h4d_set_bias(h4d_system *s, double x_b, double alpha_b) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (alpha_b > 0.0 && s->la.k > 0)
        return fail(H4D_EINVAL, "the bimodal bias and the learned proposal are exclusive");
    int rc = setup_bias(s, x_b, alpha_b);
    if (rc) return rc;
    s->p.bias_xb = x_b;
    s->p.bias_alpha = alpha_b;
    HIPC(hipMemcpy(const_cast<Box *>(s->a.box), s->box_h.data(), sizeof(Box) * s->nbox, hipMemcpyHostToDevice));
    s->drop_graphs();       // the captured launches hold the old parameters
    return H4D_OK;
}

int32_t h4d_set_early_rejection(h4d_system *s, double v_ex_edge) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (!(v_ex_edge >= 0.0 && std::isfinite(v_ex_edge))) return fail(H4D_EINVAL, "v_ex_edge must be finite and >= 0");
    if (v_ex_edge > 0.0 && s->la.k > 0)
        return fail(H4D_EINVAL, "early rejection and the learned proposal are exclusive");
    s->p.v_ex_edge = v_ex_edge;
    s->a.G.v_ex_half = 0.5 * v_ex_edge;
    s->drop_graphs();       // the captured launches hold the old parameters
    return H4D_OK;
}

int32_t h4d_set_trial_index(h4d_system *s, uint64_t trial) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    int rc = read_ctl(s);
    if (rc) return rc;
    for (int b = 0; b < s->nbox; ++b) s->h_ctl[b].trial = (long long)trial;
    return write_ctl(s);
}

static int save_box(h4d_system *s, int box, h4d_checkpoint *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    if (box < 0 || box >= s->nbox || (s->speculative && box != 0))
        return fail(H4D_EINVAL, "box index out of range (speculative handles: box 0)");
    int rc = read_ctl(s);
    if (rc) return rc;
    const Ctl &c = s->h_ctl[box];     // (replicas hold the chain's state between calls)
    const h4d_system::Stats &st = s->speculative ? s->chain : s->stats[box];
    const Box &B = s->box_h[box];
    std::memset(out, 0, sizeof(*out));
    out->params = s->p;
    for (int d = 0; d < 3; ++d) out->params.box[d] = B.L[d];   // the box's own edges and stream
    out->params.stream = B.stream;
    out->trial = (uint64_t)c.trial;
    out->md_phases = (uint64_t)c.md;
    out->next_tag = c.next_tag;
    out->lanes_per_atom = s->a.lanes;
    out->rebuild_every = s->rebuild_every;
    out->clean_trials = s->clean_trials;
    out->interval_tuned = s->interval_tuned ? 1 : 0;
    out->nbr_cap = s->a.nbr_cap;
    out->cell_cap = s->a.cell_cap;
    out->has_velocities = (s->p.momenta || s->vel_canonical) ? 1 : 0;
    out->n_trials = st.n_trials;
    out->n_ins = st.n_ins;
    out->n_ins_acc = st.n_ins_acc;
    out->n_del = st.n_del;
    out->n_del_acc = st.n_del_acc;
    out->N_sum = st.N_sum;
    out->N2_sum = st.N2_sum;
    return H4D_OK;
}

static int restore_box(h4d_system *s, int box, const h4d_checkpoint *ck, int32_t n_atoms, const double *vel) {
    if (!s || !ck) return fail(H4D_EINVAL, "null argument");
    if (box < 0 || box >= s->nbox || (s->speculative && box != 0))
        return fail(H4D_EINVAL, "box index out of range (speculative handles: box 0)");
    const h4d_params &q = ck->params;
    const Box &B0 = s->box_h[box];
    bool same_box = true;
    for (int d = 0; d < 3; ++d) same_box &= q.box[d] == B0.L[d];
    if (q.seed != s->p.seed || q.stream != B0.stream || !same_box || q.precision != s->p.precision ||
        q.momenta != s->p.momenta || q.n_types != s->p.n_types || q.water != s->p.water)
        return fail(H4D_EINVAL, "the handle was not created with the checkpoint's parameters");
    if (ck->lanes_per_atom != 4 && ck->lanes_per_atom != 8 && ck->lanes_per_atom != 16)
        return fail(H4D_EINVAL, "lanes_per_atom must be 4, 8 or 16");
    if (ck->rebuild_every < 1 || ck->clean_trials < 0 || ck->nbr_cap < 1 || ck->cell_cap < 1 ||
        ck->nbr_cap % kMaxLanes != 0)
        return fail(H4D_EINVAL, "invalid rebuild interval or list capacity");
    if (ck->has_velocities && !vel) return fail(H4D_EINVAL, "the checkpoint carries momenta: vel is required");
    int rc = read_ctl(s);
    if (rc) return rc;
    // the boxes this record applies to: every replica of a speculative
    // handle, else the one box
    const int b0 = s->speculative ? 0 : box, b1 = s->speculative ? s->nbox : box + 1;
    Ctl &c = s->h_ctl[box];
    for (int b = b0; b < b1; ++b)
        if (n_atoms != s->h_ctl[b].n) return fail(H4D_EINVAL, "n_atoms differs from the handle's state");
    long long max_tag = -1;
    if (c.n) {
        std::vector<long long> tags(c.n);
        HIPC(hipMemcpyAsync(tags.data(), s->a.ctag + s->box_h[box].a0, sizeof(long long) * c.n,
                            hipMemcpyDeviceToHost, s->stream));
        HIPC(hipStreamSynchronize(s->stream));
        for (long long t : tags) max_tag = std::max(max_tag, t);
    }
    if (ck->next_tag <= max_tag) return fail(H4D_EINVAL, "next_tag must exceed every tag of the state");
    KArgs &a = s->a;
    // list capacities as the saved handle had them (the list layout follows them)
    if (ck->nbr_cap != a.nbr_cap) {
        s->release(a.nbr);
        a.nbr_cap = ck->nbr_cap;
        if ((rc = s->alloc(&a.nbr, nbr_elems(s)))) return rc;
    }
    if (ck->cell_cap != a.cell_cap) {
        s->release(a.cell_atoms[0]);
        s->release(a.cell_atoms[1]);
        a.cell_cap = ck->cell_cap;
        if ((rc = s->alloc(&a.cell_atoms[0], (size_t)a.ncell_total * a.cell_cap))) return rc;
        if ((rc = s->alloc(&a.cell_atoms[1], (size_t)a.ncell_total * a.cell_cap))) return rc;
    }
    set_lanes(s, ck->lanes_per_atom);
    s->drop_graphs();
    s->rebuild_every = ck->rebuild_every;
    s->clean_trials = ck->clean_trials;
    s->interval_tuned = ck->interval_tuned != 0;
    if (ck->has_velocities && c.n) {
        std::vector<double4> buf(c.n);
        for (int i = 0; i < c.n; ++i) buf[i] = make_double4(vel[3 * i], vel[3 * i + 1], vel[3 * i + 2], 0.0);
        for (int b = b0; b < b1; ++b)
            HIPC(hipMemcpyAsync(a.cvel + s->box_h[b].a0, buf.data(), sizeof(double4) * c.n,
                                hipMemcpyHostToDevice, s->stream));
        HIPC(hipStreamSynchronize(s->stream));
    }
    s->vel_canonical = ck->has_velocities != 0;
    h4d_system::Stats st;
    st.n_trials = ck->n_trials;
    st.n_ins = ck->n_ins;
    st.n_ins_acc = ck->n_ins_acc;
    st.n_del = ck->n_del;
    st.n_del_acc = ck->n_del_acc;
    st.N_sum = ck->N_sum;
    st.N2_sum = ck->N2_sum;
    for (int b = b0; b < b1; ++b) {
        Ctl &cb = s->h_ctl[b];
        cb.trial = (long long)ck->trial;
        cb.md = (long long)ck->md_phases;
        cb.next_tag = ck->next_tag;
        s->stats[b] = st;
    }
    if (s->speculative) s->chain = st;
    if ((rc = write_ctl(s))) return rc;
    return h4d_build_neighbors(s);
}

int32_t h4d_save_checkpoint(h4d_system *s, h4d_checkpoint *ck) {
    if (s && s->nbox != 1 && !s->speculative)
        return fail(H4D_EINVAL, "a batch holds one chain per box: h4d_save_box_checkpoint");
    return save_box(s, 0, ck);
}

int32_t h4d_restore_checkpoint(h4d_system *s, const h4d_checkpoint *ck, int32_t n_atoms, const double *vel) {
    if (s && s->nbox != 1 && !s->speculative)
        return fail(H4D_EINVAL, "a batch holds one chain per box: h4d_restore_box_checkpoint");
    return restore_box(s, 0, ck, n_atoms, vel);
}

int32_t h4d_save_box_checkpoint(h4d_system *s, int32_t box, h4d_checkpoint *ck) { return save_box(s, box, ck); }

int32_t h4d_restore_box_checkpoint(h4d_system *s, int32_t box, const h4d_checkpoint *ck, int32_t n_atoms,
                                   const double *vel) {
    return restore_box(s, box, ck, n_atoms, vel);
}

int32_t h4d_get_state(h4d_system *s, int32_t cap, int32_t *n, int32_t *n_salt, double *pos, double *vel,
                      int32_t *type, int32_t *mol, int64_t *tag) {
    return box_state(s, 0, cap, n, n_salt, pos, vel, type, mol, tag);
}

int32_t h4d_get_box_state(h4d_system *s, int32_t box, int32_t cap, int32_t *n, int32_t *n_salt, double *pos,
                          double *vel, int32_t *type, int32_t *mol, int64_t *tag) {
    return box_state(s, box, cap, n, n_salt, pos, vel, type, mol, tag);
}

int32_t h4d_forces_at(h4d_system *s, const int32_t flying[2], double w, double *forces, double *energy) {
    if (!s || !flying) return fail(H4D_EINVAL, "null argument");
    if (s->nbox != 1) return fail(H4D_EINVAL, "the force hook serves single-box systems");
    const int n = s->n_host[0];
    for (int q = 0; q < 2; ++q)
        if (flying[q] < -1 || flying[q] >= n) return fail(H4D_EINVAL, "flying index out of range");
    KArgs &a = s->a;
    for (int q = 0; q < 2; ++q)
        if (flying[q] >= 0) hipLaunchKernelGGL(k_set_fly, dim3(1), dim3(1), 0, s->stream, a, flying[q], 1);
    int rc = h4d_build_neighbors(s);
    if (rc) return rc;
    if (s->p.precision == H4D_PREC_FP32) launch_forces<1>(s, w);
    else launch_forces<0>(s, w);
    HIPC(hipGetLastError());
    hipLaunchKernelGGL(k_energy, dim3(a.step_blocks), dim3(kBlock), 0, s->stream, a, 2, 0, w, 0);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s->stream, a, 2);
    HIPC(hipGetLastError());
    if ((rc = read_ctl(s))) return rc;
    if (forces && n) {
        std::vector<double4> buf(n);
        HIPC(hipMemcpy(buf.data(), a.force, sizeof(double4) * n, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) {
            forces[3 * i] = buf[i].x;
            forces[3 * i + 1] = buf[i].y;
            forces[3 * i + 2] = buf[i].z;
        }
    }
    if (energy) {
        energy[0] = s->h_ctl[0].Ulj + s->h_ctl[0].Uc;
        energy[1] = s->h_ctl[0].Ulj;
        energy[2] = s->h_ctl[0].Uc;
    }
    for (int q = 0; q < 2; ++q)
        if (flying[q] >= 0) hipLaunchKernelGGL(k_set_fly, dim3(1), dim3(1), 0, s->stream, a, flying[q], 0);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int32_t h4d_sample_observables(h4d_system *s, h4d_observables *out) { return box_observables(s, 0, out); }

int32_t h4d_box_observables(h4d_system *s, int32_t box, h4d_observables *out) {
    return box_observables(s, box, out);
}

int32_t h4d_set_list_loads(h4d_system *s, int32_t mode) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (mode < -1 || mode > 1) return fail(H4D_EINVAL, "list-load mode must be -1, 0 or 1");
    s->list_loads = mode;   // the round graphs are keyed by the kind in use
    return H4D_OK;
}

int32_t h4d_set_timing(h4d_system *s, int32_t on) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if ((on != 0) != s->timing) s->drop_graphs();
    s->timing = on != 0;
    s->retries = 0;
    s->step_launches = 0;
    s->step_ms = 0.0;
    s->atom_launches = 0.0;
    return H4D_OK;
}

int32_t h4d_get_timing(h4d_system *s, h4d_timing *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    unsigned long long *d = nullptr;
    int rc = s->alloc(&d, 1);
    if (rc) return rc;
    HIPC(hipMemsetAsync(d, 0, sizeof(*d), s->stream));
    hipLaunchKernelGGL(k_sum_nbr, dim3(slot_blocks(s)), dim3(kBlock), 0, s->stream, s->a, d);
    unsigned long long sum = 0;
    HIPC(hipMemcpyAsync(&sum, d, sizeof(sum), hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    s->release(d);
    long long atoms = 0;
    for (int b = 0; b < s->nbox; ++b) atoms += s->n_host[b];
    out->step_launches = s->step_launches;
    out->step_ms = s->step_ms;
    out->mean_nbr = atoms > 0 ? (double)sum / (double)atoms : 0.0;
    out->rebuild_every = s->rebuild_every;
    out->nbr_cap = s->a.nbr_cap;
    out->lanes = s->a.lanes;
    out->cell_cap = s->a.cell_cap;
    out->retries = s->retries;
    out->atom_launches = s->atom_launches;
    out->nonfinite = s->nonfinite;
    out->retries_total = s->retries_total;
    out->nt_lists = nt_lists(s) ? 1 : 0;
    out->reserved = 0;
    return H4D_OK;
}

}  // extern "C"

namespace {

// Wall time per atom-step of `trials` trials (per box) with the current
// launch shape, after one untimed round that captures its graph.
int time_shape(h4d_system *s, int trials, std::vector<h4d_trial> &recs, double *sec_per_atom_step) {
    int rc;
    if ((rc = s->nbox == 1 ? run_one(s, 0, recs.data()) : run_batch(s, 1, 0, recs.data()))) return rc;
    HIPC(hipStreamSynchronize(s->stream));
    const auto t0 = std::chrono::steady_clock::now();
    if (s->nbox == 1) {
        for (int t = 0; t < trials && !rc; ++t) rc = run_one(s, 0, recs.data() + t);
    } else {
        rc = run_batch(s, trials, 0, recs.data());
    }
    if (rc) return rc;
    HIPC(hipStreamSynchronize(s->stream));
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    double atom_steps = 0.0;
    for (const h4d_trial &r : recs) atom_steps += (double)r.n_atoms * (double)r.n_steps;
    *sec_per_atom_step = atom_steps > 0.0 ? sec / atom_steps : sec;
    return H4D_OK;
}

}  // namespace

extern "C" {

int32_t h4d_autotune(h4d_system *s, int32_t trials, int32_t *lanes_out, int32_t *rebuild_out,
                     double *ns_per_atom_step) {
    if (!s || trials < 1) return fail(H4D_EINVAL, "null handle or trials < 1");
    const int cand[3] = {4, 8, 16};
    int best = s->a.lanes;
    double best_t = 0.0;
    std::vector<h4d_trial> recs((size_t)trials * s->nbox);
    int rc;
    for (int q = 0; q < 3; ++q) {
        set_lanes(s, cand[q]);
        s->drop_graphs();
        double t = 0.0;
        if ((rc = time_shape(s, trials, recs, &t))) return rc;
        if (q == 0 || t < best_t) { best_t = t; best = cand[q]; }
    }
    set_lanes(s, best);
    s->drop_graphs();
    // blocks per cell of the list build (cell form only)
    if (s->cells && list_cells_lds(s) <= 56 * 1024) {
        const int most = std::max(1, std::min(16, s->a.cell_cap / s->list_units / (2 * kListWaves)));
        int best_split = list_split(s);
        double best_st = 0.0;
        bool first = true;
        for (int sp : {1, 2, 4, 8, 16}) {
            if (sp > most) break;
            s->list_split = sp;
            s->drop_graphs();
            double t = 0.0;
            if ((rc = time_shape(s, trials, recs, &t))) return rc;
            if (first || t < best_st) { best_st = t; best_split = sp; first = false; }
        }
        s->list_split = best_split;
        s->drop_graphs();
        if (!first) best_t = best_st;
    }
    // the base rebuild interval (unless the parameters fix it): multiples of
    // the automatic one, each timed; the best is kept for the handle's life
    if (s->p.rebuild_every == 0) {
        const int m0 = std::max(1, s->rebuild_every);
        std::vector<int> ms;
        for (int num : {1, 2, 3, 4, 6, 8})
            for (int m : {std::max(1, (m0 * num) / 4)})
                if (std::find(ms.begin(), ms.end(), m) == ms.end()) ms.push_back(m);
        int best_m = m0;
        double best_mt = 0.0;
        s->interval_tuned = true;
        for (size_t q = 0; q < ms.size(); ++q) {
            s->rebuild_every = ms[q];
            double t = 0.0;
            if ((rc = time_shape(s, trials, recs, &t))) return rc;
            if (q == 0 || t < best_mt) { best_mt = t; best_m = ms[q]; }
        }
        s->rebuild_every = best_m;
        best_t = best_mt;
    }
    s->drop_graphs();
    if ((rc = h4d_build_neighbors(s))) return rc;
    if (lanes_out) *lanes_out = best;
    if (rebuild_out) *rebuild_out = s->rebuild_every;
    if (ns_per_atom_step) *ns_per_atom_step = best_t * 1e9;
    return H4D_OK;
}

}  // extern "C"

// ==========================================================================
// Learned proposal: the network handle and its training.
// ==========================================================================
// Workspace of the network forward that allocates nothing
// (h4d_mlp_forward_static): the FP32 hidden activations of up to
// kStaticRows rows, two ping-pong layers of kStaticRows x 128 floats (4 MiB).
// Each device holds its own copy until the process ends; host code reaches it
// only through the address hipGetSymbolAddress gives on that device.
constexpr int kStaticRows = 4096;
static __device__ __align__(256) float scratch[2 * kStaticRows * kHid];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev, resolved once per device with
// that device current.
int scratch_address(int dev, float **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(H4D_ENODEV, "device index beyond the workspace table");
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        HIPC(hipGetDevice(&cur));
        if (cur != dev) HIPC(hipSetDevice(dev));
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return fail(H4D_EHIP, std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return H4D_OK;
}

}  // namespace

struct h4d_mlp {
    hipStream_t stream = nullptr;
    int device = 0;                        // the device the parameters live on
    float *scratch = nullptr;              // that device's static workspace
    float *theta = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    bf16x4 *wfrag = nullptr;
    long long adam_t = 0;
    int rows = 0;                          // capacity of the activation buffers
    float *X = nullptr, *T = nullptr, *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Z3 = nullptr,
          *A3 = nullptr, *Sz = nullptr, *S = nullptr, *dS = nullptr, *dZ3 = nullptr, *dZ2 = nullptr,
          *dZ1 = nullptr, *loss = nullptr;
    std::vector<void *> act;
    ~h4d_mlp() {
        for (void *q : act) (void)hipFree(q);
        for (void *q : {(void *)theta, (void *)m, (void *)v, (void *)g, (void *)wfrag}) if (q) (void)hipFree(q);
    }
};

namespace {

int mlp_rows(h4d_mlp *n, int rows) {
    if (rows <= n->rows) return H4D_OK;
    for (void *q : n->act) (void)hipFree(q);
    n->act.clear();
    auto get = [&](float **p, size_t cnt) -> int {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(cnt, 1) * sizeof(float)) != hipSuccess)
            return fail(H4D_ENOMEM, "hipMalloc of network activations failed");
        n->act.push_back(q);
        *p = static_cast<float *>(q);
        return H4D_OK;
    };
    const size_t R = (size_t)rows;
    int rc;
    if ((rc = get(&n->X, R * kFeat)) || (rc = get(&n->T, R)) || (rc = get(&n->Z1, R * kHid)) ||
        (rc = get(&n->A1, R * kHid)) || (rc = get(&n->Z2, R * kHid)) || (rc = get(&n->A2, R * kHid)) ||
        (rc = get(&n->Z3, R * kHid)) || (rc = get(&n->A3, R * kHid)) || (rc = get(&n->Sz, R)) ||
        (rc = get(&n->S, R)) || (rc = get(&n->dS, R)) || (rc = get(&n->dZ3, R * kHid)) ||
        (rc = get(&n->dZ2, R * kHid)) || (rc = get(&n->dZ1, R * kHid)) || (rc = get(&n->loss, 1)))
        return rc;
    n->rows = rows;
    return H4D_OK;
}

int mlp_pack(h4d_mlp *n) {
    const int nf = kFragL1 + 2 * kFragL2;
    hipLaunchKernelGGL(k_mlp_pack, dim3(blocks_for(nf)), dim3(kBlock), 0, n->stream, n->theta, n->wfrag);
    HIPC(hipGetLastError());
    return H4D_OK;
}

// FP32 forward of rows X[0..rows) (logits in S)
void mlp_fwd32(h4d_mlp *n, int rows) {
    const hipStream_t st = n->stream;
    const float *th = n->theta;
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->X, th + kOffW1,
                       th + kOffB1, n->Z1, n->A1, rows, kFeat, kHid, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->A1, th + kOffW2,
                       th + kOffB2, n->Z2, n->A2, rows, kHid, kHid, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->A2, th + kOffW3,
                       th + kOffB3, n->Z3, n->A3, rows, kHid, kHid, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for(rows)), dim3(kBlock), 0, st, n->A3, th + kOffW4, th + kOffB4,
                       n->Sz, n->S, rows, kHid, 1, 0);
}

// loss of S against T and the gradient of the mean loss into g
void mlp_bwd32(h4d_mlp *n, int rows) {
    const hipStream_t st = n->stream;
    const float *th = n->theta;
    float *g = n->g;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, n->S, n->T, rows, n->dS, n->loss);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks_for((kHid + 1) * 1)), dim3(kBlock), 0, st, n->A3, n->dS, rows, kHid, 1,
                       g + kOffW4, g + kOffB4);
    hipLaunchKernelGGL(k_dgrad, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->dS, th + kOffW4, n->Z3, rows,
                       kHid, 1, n->dZ3);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks_for((kHid + 1) * kHid)), dim3(kBlock), 0, st, n->A2, n->dZ3, rows, kHid,
                       kHid, g + kOffW3, g + kOffB3);
    hipLaunchKernelGGL(k_dgrad, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->dZ3, th + kOffW3, n->Z2, rows,
                       kHid, kHid, n->dZ2);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks_for((kHid + 1) * kHid)), dim3(kBlock), 0, st, n->A1, n->dZ2, rows, kHid,
                       kHid, g + kOffW2, g + kOffB2);
    hipLaunchKernelGGL(k_dgrad, dim3(blocks_for(rows * kHid)), dim3(kBlock), 0, st, n->dZ2, th + kOffW2, n->Z1, rows,
                       kHid, kHid, n->dZ1);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks_for((kFeat + 1) * kHid)), dim3(kBlock), 0, st, n->X, n->dZ1, rows, kFeat,
                       kHid, g + kOffW1, g + kOffB1);
}

uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int32_t h4d_mlp_create(uint64_t seed, void *hip_stream, h4d_mlp **out) {
    g_err.clear();
    if (!out) return fail(H4D_EINVAL, "null argument");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(H4D_ENODEV, "no HIP device");
    auto *n = new h4d_mlp();
    n->stream = static_cast<hipStream_t>(hip_stream);
    int rc0 = hipGetDevice(&n->device) == hipSuccess ? scratch_address(n->device, &n->scratch)
                                                     : fail(H4D_EHIP, "hipGetDevice failed");
    if (rc0) { delete n; return rc0; }
    const size_t P = kParams;
    if (hipMalloc((void **)&n->theta, P * 4) != hipSuccess || hipMalloc((void **)&n->m, P * 4) != hipSuccess ||
        hipMalloc((void **)&n->v, P * 4) != hipSuccess || hipMalloc((void **)&n->g, P * 4) != hipSuccess ||
        hipMalloc((void **)&n->wfrag, sizeof(bf16x4) * (kFragL1 + 2 * kFragL2)) != hipSuccess) {
        delete n;
        return fail(H4D_ENOMEM, "hipMalloc of network parameters failed");
    }
    // Glorot-uniform weights, zero biases, from a seeded splitmix64 stream
    std::vector<float> th(P, 0.0f);
    uint64_t x = seed;
    const int fan[4][3] = {{kOffW1, kFeat, kHid}, {kOffW2, kHid, kHid}, {kOffW3, kHid, kHid}, {kOffW4, kHid, 1}};
    for (const auto &f : fan) {
        const double lim = std::sqrt(6.0 / (f[1] + f[2]));
        for (int q = 0; q < f[1] * f[2]; ++q) {
            const double u = ((double)(splitmix64(x) >> 11) + 0.5) * 0x1p-53;
            th[f[0] + q] = (float)(lim * (2.0 * u - 1.0));
        }
    }
    if (hipMemcpy(n->theta, th.data(), P * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, P * 4) != hipSuccess || hipMemset(n->v, 0, P * 4) != hipSuccess) {
        delete n;
        return fail(H4D_EHIP, "network upload failed");
    }
    int rc = mlp_pack(n);
    if (rc) { delete n; return rc; }
    *out = n;
    return H4D_OK;
}

int32_t h4d_mlp_destroy(h4d_mlp *n) {
    if (!n) return H4D_OK;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    delete n;
    return H4D_OK;
}

int32_t h4d_mlp_set_weights(h4d_mlp *n, const float *theta) {
    if (!n || !theta) return fail(H4D_EINVAL, "null argument");
    HIPC(hipMemcpyAsync(n->theta, theta, sizeof(float) * kParams, hipMemcpyHostToDevice, n->stream));
    HIPC(hipMemsetAsync(n->m, 0, sizeof(float) * kParams, n->stream));
    HIPC(hipMemsetAsync(n->v, 0, sizeof(float) * kParams, n->stream));
    n->adam_t = 0;
    int rc = mlp_pack(n);
    if (rc) return rc;
    HIPC(hipStreamSynchronize(n->stream));
    return H4D_OK;
}

int32_t h4d_mlp_get_weights(h4d_mlp *n, float *theta) {
    if (!n || !theta) return fail(H4D_EINVAL, "null argument");
    HIPC(hipMemcpyAsync(theta, n->theta, sizeof(float) * kParams, hipMemcpyDeviceToHost, n->stream));
    HIPC(hipStreamSynchronize(n->stream));
    return H4D_OK;
}

int32_t h4d_mlp_forward(h4d_mlp *n, int32_t rows, const float *features, int32_t bf16, float *logits) {
    if (!n || rows < 0 || (rows && (!features || !logits))) return fail(H4D_EINVAL, "null argument or negative size");
    if (!rows) return H4D_OK;
    int rc = mlp_rows(n, rows);
    if (rc) return rc;
    HIPC(hipMemcpyAsync(n->X, features, sizeof(float) * rows * kFeat, hipMemcpyHostToDevice, n->stream));
    if (bf16) hipLaunchKernelGGL(k_mlp_infer, dim3((rows + 63) / 64), dim3(256), 0, n->stream, n->X, rows, n->theta,
                                 n->wfrag, n->S);
    else mlp_fwd32(n, rows);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(logits, n->S, sizeof(float) * rows, hipMemcpyDeviceToHost, n->stream));
    HIPC(hipStreamSynchronize(n->stream));
    return H4D_OK;
}

int32_t h4d_mlp_forward_static(h4d_mlp *n, int32_t rows, const float *features, int32_t bf16, float *logits) {
    if (!n || rows < 0 || (rows && (!features || !logits))) return fail(H4D_EINVAL, "null argument or negative size");
    if (rows > kStaticRows)
        return fail(H4D_EINVAL, "rows exceed the static workspace (at most " + std::to_string(kStaticRows) + ")");
    if (!rows) return H4D_OK;
    int cur = -1;
    HIPC(hipGetDevice(&cur));
    if (cur != n->device) return fail(H4D_EINVAL, "call on the device the network was created on");
    const hipStream_t st = n->stream;
    const float *th = n->theta;
    if (bf16) {
        hipLaunchKernelGGL(k_mlp_infer, dim3((rows + 63) / 64), dim3(256), 0, st, features, rows, th, n->wfrag,
                           logits);
    } else {   // the FP32 forward of mlp_fwd32, activations ping-ponged through the workspace
        float *h0 = n->scratch, *h1 = n->scratch + (size_t)kStaticRows * kHid;
        const dim3 grid(blocks_for(rows * kHid));
        hipLaunchKernelGGL(k_dense_fwd, grid, dim3(kBlock), 0, st, features, th + kOffW1, th + kOffB1, nullptr, h0,
                           rows, kFeat, kHid, 1);
        hipLaunchKernelGGL(k_dense_fwd, grid, dim3(kBlock), 0, st, h0, th + kOffW2, th + kOffB2, nullptr, h1, rows,
                           kHid, kHid, 1);
        hipLaunchKernelGGL(k_dense_fwd, grid, dim3(kBlock), 0, st, h1, th + kOffW3, th + kOffB3, nullptr, h0, rows,
                           kHid, kHid, 1);
        hipLaunchKernelGGL(k_dense_fwd, dim3(blocks_for(rows)), dim3(kBlock), 0, st, h0, th + kOffW4, th + kOffB4,
                           nullptr, logits, rows, kHid, 1, 0);
    }
    HIPC(hipGetLastError());
    return H4D_OK;
}

int32_t h4d_mlp_loss_grad(h4d_mlp *n, int32_t rows, const float *features, const float *targets, float *grad,
                          float *loss) {
    if (!n || rows < 1 || !features || !targets) return fail(H4D_EINVAL, "null argument or rows < 1");
    int rc = mlp_rows(n, rows);
    if (rc) return rc;
    HIPC(hipMemcpyAsync(n->X, features, sizeof(float) * rows * kFeat, hipMemcpyHostToDevice, n->stream));
    HIPC(hipMemcpyAsync(n->T, targets, sizeof(float) * rows, hipMemcpyHostToDevice, n->stream));
    mlp_fwd32(n, rows);
    mlp_bwd32(n, rows);
    HIPC(hipGetLastError());
    if (grad) HIPC(hipMemcpyAsync(grad, n->g, sizeof(float) * kParams, hipMemcpyDeviceToHost, n->stream));
    if (loss) HIPC(hipMemcpyAsync(loss, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    HIPC(hipStreamSynchronize(n->stream));
    return H4D_OK;
}

int32_t h4d_mlp_train(h4d_mlp *n, int32_t rows, const float *features, const float *targets, int32_t steps,
                      int32_t batch, float lr, float weight_decay, uint64_t seed, float *losses) {
    if (!n || rows < 1 || !features || !targets || steps < 0 || batch < 1 || !(lr > 0.0f) || !(weight_decay >= 0.0f))
        return fail(H4D_EINVAL, "bad training arguments");
    batch = std::min(batch, rows);
    int rc = mlp_rows(n, batch);
    if (rc) return rc;
    float *data = nullptr, *tg = nullptr, *lossv = nullptr;
    int *idx = nullptr;
    auto cleanup = [&]() {
        if (data) (void)hipFree(data);
        if (tg) (void)hipFree(tg);
        if (lossv) (void)hipFree(lossv);
        if (idx) (void)hipFree(idx);
    };
    if (hipMalloc((void **)&data, sizeof(float) * rows * kFeat) != hipSuccess ||
        hipMalloc((void **)&tg, sizeof(float) * rows) != hipSuccess ||
        hipMalloc((void **)&lossv, sizeof(float) * std::max(1, steps)) != hipSuccess ||
        hipMalloc((void **)&idx, sizeof(int) * (size_t)std::max(1, steps) * batch) != hipSuccess) {
        cleanup();
        return fail(H4D_ENOMEM, "hipMalloc of training data failed");
    }
    // the network trains on standardized features (mean 0, variance 1 per
    // column over the data); the affine map is folded into the first layer
    // afterwards, so the stored network reads raw features
    std::vector<double> mean(kFeat, 0.0), sdev(kFeat, 0.0);
    for (int r = 0; r < rows; ++r)
        for (int q = 0; q < kFeat; ++q) mean[q] += features[(size_t)r * kFeat + q];
    for (int q = 0; q < kFeat; ++q) mean[q] /= rows;
    for (int r = 0; r < rows; ++r)
        for (int q = 0; q < kFeat; ++q) {
            const double d = features[(size_t)r * kFeat + q] - mean[q];
            sdev[q] += d * d;
        }
    for (int q = 0; q < kFeat; ++q) {
        sdev[q] = std::sqrt(sdev[q] / rows);
        if (!(sdev[q] > 1e-6)) sdev[q] = 1.0;
    }
    std::vector<float> stdX((size_t)rows * kFeat);
    for (int r = 0; r < rows; ++r)
        for (int q = 0; q < kFeat; ++q)
            stdX[(size_t)r * kFeat + q] = (float)((features[(size_t)r * kFeat + q] - mean[q]) / sdev[q]);
    std::vector<float> th(kParams);
    if (hipMemcpy(th.data(), n->theta, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return fail(H4D_EHIP, "network download failed");
    }
    // the current network in standardized coordinates: W1' = sd W1, b1' = b1 + mean W1
    for (int o = 0; o < kHid; ++o) {
        double b = th[kOffB1 + o];
        for (int q = 0; q < kFeat; ++q) b += mean[q] * th[kOffW1 + q * kHid + o];
        th[kOffB1 + o] = (float)b;
    }
    for (int q = 0; q < kFeat; ++q)
        for (int o = 0; o < kHid; ++o) th[kOffW1 + q * kHid + o] = (float)(th[kOffW1 + q * kHid + o] * sdev[q]);
    if (hipMemcpy(n->theta, th.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return fail(H4D_EHIP, "network upload failed");
    }
    features = stdX.data();
    // minibatches: consecutive slices of seeded shuffles of the rows
    std::vector<int> order(rows), all((size_t)std::max(1, steps) * batch);
    for (int r = 0; r < rows; ++r) order[r] = r;
    std::mt19937_64 gen(seed);
    int pos = rows;
    for (int q = 0; q < steps; ++q)
        for (int b = 0; b < batch; ++b) {
            if (pos == rows) { std::shuffle(order.begin(), order.end(), gen); pos = 0; }
            all[(size_t)q * batch + b] = order[pos++];
        }
    const hipStream_t st = n->stream;
    bool ok = hipMemcpyAsync(data, features, sizeof(float) * rows * kFeat, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(tg, targets, sizeof(float) * rows, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(idx, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int q = 0; ok && q < steps; ++q) {
        hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(batch * kFeat)), dim3(kBlock), 0, st, data, tg,
                           idx + (size_t)q * batch, batch, n->X, n->T);
        mlp_fwd32(n, batch);
        mlp_bwd32(n, batch);
        ok = hipMemcpyAsync(lossv + q, n->loss, sizeof(float), hipMemcpyDeviceToDevice, st) == hipSuccess;
        n->adam_t += 1;
        const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)n->adam_t)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)n->adam_t)));
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams)), dim3(kBlock), 0, st, n->theta, n->m, n->v, n->g,
                           kParams, lr, b1, b2, eps, c1, c2, weight_decay);
    }
    ok = ok && hipGetLastError() == hipSuccess;
    if (ok && losses && steps)
        ok = hipMemcpyAsync(losses, lossv, sizeof(float) * steps, hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    cleanup();
    if (!ok) return fail(H4D_EHIP, "network training failed");
    // back to raw features: W1 = W1' / sd, b1 = b1' - (mean / sd) W1'
    if (hipMemcpy(th.data(), n->theta, sizeof(float) * kParams, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(H4D_EHIP, "network download failed");
    for (int o = 0; o < kHid; ++o) {
        double b = th[kOffB1 + o];
        for (int q = 0; q < kFeat; ++q) b -= mean[q] / sdev[q] * th[kOffW1 + q * kHid + o];
        th[kOffB1 + o] = (float)b;
    }
    for (int q = 0; q < kFeat; ++q)
        for (int o = 0; o < kHid; ++o) th[kOffW1 + q * kHid + o] = (float)(th[kOffW1 + q * kHid + o] / sdev[q]);
    if (hipMemcpy(n->theta, th.data(), sizeof(float) * kParams, hipMemcpyHostToDevice) != hipSuccess)
        return fail(H4D_EHIP, "network upload failed");
    // Adam's moments belong to the standardized coordinates: start afresh
    if (hipMemset(n->m, 0, sizeof(float) * kParams) != hipSuccess ||
        hipMemset(n->v, 0, sizeof(float) * kParams) != hipSuccess)
        return fail(H4D_EHIP, "optimiser reset failed");
    n->adam_t = 0;
    return mlp_pack(n);
}

int32_t h4d_set_proposal(h4d_system *s, const h4d_mlp *net, int32_t k, double logit_cap, double weight_scale) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (!(logit_cap == logit_cap) || !std::isfinite(weight_scale) || weight_scale < 0.0)
        return fail(H4D_EINVAL, "logit_cap must not be NaN and weight_scale must be finite and >= 0");
    if (k > 65536) return fail(H4D_EINVAL, "at most 65536 candidates");
    if (k > 0 && (int64_t)k * s->nbox * 2 * kWave > (int64_t)INT32_MAX)
        return fail(H4D_EINVAL, "candidates times boxes too large");
    if (k > 0 && s->a.G.bias_alpha > 0.0)
        return fail(H4D_EINVAL, "the bimodal bias and the learned proposal are exclusive");
    if (k > 0 && s->a.G.v_ex_half > 0.0)
        return fail(H4D_EINVAL, "early rejection and the learned proposal are exclusive");
    s->drop_graphs();
    LearnArgs &l = s->la;
    for (void *q : {(void *)l.sites, (void *)l.feat, (void *)l.logit}) if (q) s->release(q);
    l.sites = nullptr; l.feat = nullptr; l.logit = nullptr;
    l.k = 0;
    l.use_net = 0;
    if (k <= 0) return H4D_OK;
    int rc;
    const size_t rows = (size_t)k * s->nbox;   // every box has its own candidates
    if ((rc = s->alloc(&l.sites, 6 * rows)) || (rc = s->alloc(&l.feat, (size_t)kFeat * rows)) ||
        (rc = s->alloc(&l.logit, rows)))
        return rc;
    if (!l.last_feat) {
        if ((rc = s->alloc(&l.last_feat, (size_t)kFeat * s->nbox))) return rc;
        HIPC(hipMemset(l.last_feat, 0, sizeof(float) * kFeat * s->nbox));
    }
    l.k = k;
    l.cap = logit_cap;
    l.scale = weight_scale;
    l.use_net = net != nullptr;
    l.theta = net ? net->theta : nullptr;
    l.wfrag = net ? net->wfrag : nullptr;
    return H4D_OK;
}

int32_t h4d_last_site_features(h4d_system *s, float *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    if (!s->la.last_feat) return fail(H4D_EINVAL, "no learned-proposal trial has run");
    HIPC(hipMemcpyAsync(out, s->la.last_feat, sizeof(float) * kFeat, hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int32_t h4d_last_box_candidates(h4d_system *s, int32_t box, int32_t cap, double *sites, float *features,
                                float *logits) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (box < 0 || box >= s->nbox) return fail(H4D_EINVAL, "box index out of range");
    const int k = s->la.k;
    if (k <= 0) return fail(H4D_EINVAL, "the uniform proposal has no candidates");
    if (cap < k) return fail(H4D_EINVAL, "cap smaller than the number of candidates");
    const size_t g0 = (size_t)box * k;
    if (sites)
        HIPC(hipMemcpyAsync(sites, s->la.sites + 6 * g0, sizeof(double) * 6 * k, hipMemcpyDeviceToHost, s->stream));
    if (features)
        HIPC(hipMemcpyAsync(features, s->la.feat + kFeat * g0, sizeof(float) * kFeat * k, hipMemcpyDeviceToHost,
                            s->stream));
    if (logits) HIPC(hipMemcpyAsync(logits, s->la.logit + g0, sizeof(float) * k, hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return k;
}

int32_t h4d_last_candidates(h4d_system *s, int32_t cap, double *sites, float *features, float *logits) {
    return h4d_last_box_candidates(s, 0, cap, sites, features, logits);
}

int32_t h4d_site_features(h4d_system *s, int32_t n, const double *sites, float *features) {
    if (!s || n < 1 || !sites || !features) return fail(H4D_EINVAL, "null argument or n < 1");
    if (s->nbox != 1) return fail(H4D_EINVAL, "site features serve single-box systems");
    int rc = h4d_build_neighbors(s);
    if (rc) return rc;
    LearnArgs l = s->la;
    double *sd = nullptr;
    float *fd = nullptr;
    if ((rc = s->alloc(&sd, (size_t)6 * n)) || (rc = s->alloc(&fd, (size_t)kFeat * n))) return rc;
    l.k = n;
    l.sites = sd;
    l.feat = fd;
    HIPC(hipMemcpyAsync(sd, sites, sizeof(double) * 6 * n, hipMemcpyHostToDevice, s->stream));
    // the current state is an N-state for this hook: evaluated as the
    // insertion phase does (the hook's kernel takes no move flag)
    hipLaunchKernelGGL(k_site_features_hook, dim3((2 * n * kWave + kBlock - 1) / kBlock), dim3(kBlock), 0, s->stream,
                       s->a, l);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(features, fd, sizeof(float) * kFeat * n, hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    s->release(sd);
    s->release(fd);
    return H4D_OK;
}

}  // extern "C"

namespace {
__global__ __launch_bounds__(kBlock) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                        size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = src[i];
}
}  // namespace

extern "C" {

int32_t h4d_stream_copy(int64_t bytes, int32_t reps, double *ms) {
    if (bytes <= 0 || bytes % 16 || reps < 1 || !ms) return fail(H4D_EINVAL, "bytes must be a positive multiple of 16");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(H4D_ENODEV, "no HIP device");
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return fail(H4D_ENOMEM, "hipMalloc failed");
    if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipFree(a); return fail(H4D_ENOMEM, "hipMalloc failed"); }
    const size_t n = (size_t)bytes / 16;
    const int grid = (int)std::min<size_t>((n + kBlock - 1) / kBlock, 256 * 64);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipMemset(a, 1, bytes);
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kBlock), 0, nullptr, (const uint4 *)a, (uint4 *)b, n);
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kBlock), 0, nullptr, (const uint4 *)a, (uint4 *)b, n);
    (void)hipEventRecord(e1, nullptr);
    const hipError_t e = hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(H4D_EHIP, std::string("stream copy: ") + hipGetErrorString(e));
    *ms = t / reps;
    return H4D_OK;
}

int32_t h4d_destroy(h4d_system *s) {
    if (!s) return H4D_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    delete s;
    return H4D_OK;
}

}  // extern "C"
