// h4d_runtime.hip -- host side of the C ABI declared in include/h4d.h.
//
// Owns the device buffers of a system, enqueues the kernels of each trial
// on the caller's stream, and reads back one small record per trial (the
// only synchronisation of a trial).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "h4d.h"
#include "h4d_kernels.hpp"

using namespace h4d;

static_assert(sizeof(TrialRec) == sizeof(h4d_trial), "record layout");

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
    int cap = 0;
    int n_host = 0, nsalt_host = 0, n_mol = 0;
    int rebuild_every = 1;
    int clean_trials = 0;
    int partial_blocks = 0;
    TrialRec *h_rec = nullptr;
    Ctl *h_ctl = nullptr;
    // step-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int64_t step_launches = 0;
    double step_ms = 0.0;
    int trial_rebuilds = 0;
    int64_t retries = 0;
    int trial_M = 1;            // rebuild interval of the trial being run
    int cl = 0;                 // cell buffer of the current list (the next binning uses cl ^ 1)
    // captured trial graphs, keyed by launch shape; dropped when buffers move
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int, int, int, int, int>, hipGraphExec_t> graphs;
    bool graphs_ok[2] = {true, false};  // timed trials launch eagerly (events per step kernel)
    int last_buf = 0;           // working buffer that holds the last trajectory's end
    std::vector<void *> allocs;
    // running statistics (Eq. 1)
    int64_t n_trials = 0, n_ins = 0, n_ins_acc = 0, n_del = 0, n_del_acc = 0;
    double N_sum = 0.0, N2_sum = 0.0;

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
    const double rc = std::max(p.rc_lj, p.rc_coul);
    for (int d = 0; d < 3; ++d)
        if (!(p.box[d] >= 2.0 * rc))
            return fail(H4D_EINVAL, "every box edge must be at least twice the largest cutoff");
    if (p.water && !(p.d_oh > 0.0 && p.d_hh > 0.0 && p.d_hh < 2.0 * p.d_oh))
        return fail(H4D_EINVAL, "rigid water needs 0 < d_hh < 2 d_oh");
    return H4D_OK;
}

void setup_geo(h4d_system *s) {
    const h4d_params &p = s->p;
    Geo &G = s->a.G;
    const double two32 = 4294967296.0;
    for (int d = 0; d < 3; ++d) {
        G.L[d] = p.box[d];
        G.fx_inv[d] = two32 / p.box[d];
        G.fx_scale[d] = (float)(p.box[d] / two32);
    }
    const double rc = std::max(p.rc_lj, p.rc_coul);
    const double rlist = rc + p.skin;
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
    G.kappa = p.kappa_sr;
    G.volume = p.box[0] * p.box[1] * p.box[2];
    G.lambda3 = p.lambda_s * p.lambda_s * p.lambda_s;
    G.beta = 1.0 / p.kT;
    G.beta_mu = p.beta_mu;
    G.use_cells = 1;
    for (int d = 0; d < 3; ++d) {
        G.ncell[d] = (int)std::floor(p.box[d] / rlist);
        if (G.ncell[d] < 3) G.use_cells = 0;
    }
    if (!G.use_cells) G.ncell[0] = G.ncell[1] = G.ncell[2] = 1;
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

// Neighbour and cell capacities from the density (grown on overflow).
void initial_capacities(h4d_system *s, int n) {
    const h4d_params &p = s->p;
    const double V = p.box[0] * p.box[1] * p.box[2];
    const double rho = std::max(1.0, (double)n) / V;
    const double rlist = std::max(p.rc_lj, p.rc_coul) + p.skin;
    const double nb = 4.18879020478639 * rlist * rlist * rlist * rho;
    int cap = (int)(1.5 * nb) + 32;
    cap = std::min(cap, s->cap + kMaxLanes);
    s->a.nbr_cap = (cap + kMaxLanes - 1) / kMaxLanes * kMaxLanes;
    const Geo &G = s->a.G;
    const double cell_vol = V / ((double)G.ncell[0] * G.ncell[1] * G.ncell[2]);
    int cc = (int)(1.6 * rho * cell_vol) + 16;
    s->a.cell_cap = G.use_cells ? std::min(cc, std::max(32, s->cap)) : s->cap;
    s->a.ncell_total = G.ncell[0] * G.ncell[1] * G.ncell[2];
}

size_t nbr_elems(const h4d_system *s) {
    const int A = kWave / s->a.lanes;
    const size_t groups = (size_t)(s->cap + A - 1) / A;
    return groups * (size_t)(s->a.nbr_cap / s->a.lanes) * kWave;
}

int alloc_lists(h4d_system *s) {
    int rc;
    if ((rc = s->alloc(&s->a.nbr, nbr_elems(s)))) return rc;
    for (int q = 0; q < 2; ++q) {
        if ((rc = s->alloc(&s->a.cell_cnt[q], (size_t)s->a.ncell_total))) return rc;
        if ((rc = s->alloc(&s->a.cell_atoms[q], (size_t)s->a.ncell_total * s->a.cell_cap))) return rc;
        HIPC(hipMemset(s->a.cell_cnt[q], 0, sizeof(int) * s->a.ncell_total));
    }
    if ((rc = s->alloc(&s->a.cell_off, (size_t)s->a.ncell_total + 1))) return rc;
    if ((rc = s->alloc(&s->a.fast, (size_t)3 * kFastCap))) return rc;
    return H4D_OK;
}

int atom_blocks_l(int n, int lanes) { return std::max(1, (n * lanes + kBlock - 1) / kBlock); }

size_t list_cells_lds(const h4d_system *s) { return (size_t)s->a.cell_cap * 27 * sizeof(uint4); }

void launch_list(h4d_system *s, int b, int cb, int n_all_max, hipStream_t st) {
    KArgs &a = s->a;
    if (a.G.use_cells && list_cells_lds(s) <= 56 * 1024)
        hipLaunchKernelGGL(k_list_cells, dim3(a.ncell_total), dim3(kBlock), list_cells_lds(s), st, a, b, cb);
    else if (a.G.use_cells)
        hipLaunchKernelGGL(k_list_lanes, dim3(atom_blocks_l(n_all_max, a.lanes)), dim3(kBlock), 0, st, a, b, cb);
    else
        hipLaunchKernelGGL(k_list_allpairs, dim3(atom_blocks_l(n_all_max, a.lanes)), dim3(kBlock), 0, st, a, b, cb);
}

template <int PREC, int L>
void launch_step_l(h4d_system *s, hipStream_t st, int G, hipEvent_t e0, hipEvent_t e1, int k, int b, int bin) {
    KArgs &a = s->a;
    if (e0) hipExtLaunchKernelGGL(k_step<PREC, L>, dim3(G), dim3(kBlock), 0, st, e0, e1, 0, a, k, b, bin, s->cl);
    else hipLaunchKernelGGL((k_step<PREC, L>), dim3(G), dim3(kBlock), 0, st, a, k, b, bin, s->cl);
}

template <int PREC>
void launch_step(h4d_system *s, hipStream_t st, int G, hipEvent_t e0, hipEvent_t e1, int k, int b, int bin) {
    switch (s->a.lanes) {
        case 4: launch_step_l<PREC, 4>(s, st, G, e0, e1, k, b, bin); break;
        case 8: launch_step_l<PREC, 8>(s, st, G, e0, e1, k, b, bin); break;
        default: launch_step_l<PREC, 16>(s, st, G, e0, e1, k, b, bin); break;
    }
}

template <int PREC>
void launch_forces(h4d_system *s, int G, double w) {
    KArgs &a = s->a;
    switch (a.lanes) {
        case 4: hipLaunchKernelGGL((k_forces<PREC, 4>), dim3(G), dim3(kBlock), 0, s->stream, a, w); break;
        case 8: hipLaunchKernelGGL((k_forces<PREC, 8>), dim3(G), dim3(kBlock), 0, s->stream, a, w); break;
        default: hipLaunchKernelGGL((k_forces<PREC, 16>), dim3(G), dim3(kBlock), 0, s->stream, a, w); break;
    }
}

// Sort the canonical atoms into cell order (working buffer 0), draw the
// momenta of the current trial index, and build the list (cell buffer 0).
int sort_in(h4d_system *s, int n_all_max, hipStream_t st) {
    KArgs &a = s->a;
    const int G1 = blocks_for(n_all_max);
    const int nc = a.ncell_total;
    hipLaunchKernelGGL(k_cell_clear, dim3(blocks_for(nc)), dim3(kBlock), 0, st, a, 0);
    hipLaunchKernelGGL(k_bin_canonical, dim3(G1), dim3(kBlock), 0, st, a, 0);
    hipLaunchKernelGGL(k_cell_sort, dim3(nc), dim3(kWave), a.cell_cap * sizeof(int), st, a, 0);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, st, a, 0);
    hipLaunchKernelGGL(k_gather_in, dim3(nc), dim3(kWave), 0, st, a, 0);
    if (a.G.water) hipLaunchKernelGGL(k_rattle_mb, dim3(blocks_for(a.G.n_mol)), dim3(kBlock), 0, st, a);
    launch_list(s, 0, 0, n_all_max, st);
    s->cl = 0;
    HIPC(hipGetLastError());
    return H4D_OK;
}

// Mid-trajectory rebuild: the preceding step binned the atoms into cell
// buffer cl ^ 1.
int rebuild_mid(h4d_system *s, int b, int n_all_max, hipStream_t st) {
    KArgs &a = s->a;
    const int cb = s->cl ^ 1;
    if (a.G.use_cells)
        hipLaunchKernelGGL(k_cell_sort, dim3(a.ncell_total), dim3(kWave), a.cell_cap * sizeof(int), st, a, cb);
    launch_list(s, b, cb, n_all_max, st);
    s->cl = cb;
    HIPC(hipGetLastError());
    return H4D_OK;
}

int read_ctl(h4d_system *s) {
    HIPC(hipMemcpyAsync(s->h_ctl, s->a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int clear_errors(h4d_system *s) {
    Ctl *c = s->h_ctl;
    c->err = 0;
    c->retry = 0;
    c->max_nbr = 0;
    c->max_cell = 0;
    HIPC(hipMemcpyAsync(s->a.ctl, c, sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

// Grow the list storage after an overflow.
int grow_lists(h4d_system *s, unsigned err) {
    KArgs &a = s->a;
    const Ctl *c = s->h_ctl;
    if (err & kErrNbr) {
        int need = std::max(c->max_nbr, a.nbr_cap + kMaxLanes);
        need = (int)(need * 1.25) + kMaxLanes;
        need = (need + kMaxLanes - 1) / kMaxLanes * kMaxLanes;
        s->release(a.nbr);
        a.nbr_cap = need;
        int rc = s->alloc(&a.nbr, nbr_elems(s));
        if (rc) return rc;
    }
    if (err & kErrCell) {
        int need = std::max(c->max_cell, a.cell_cap + 8);
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

// Enqueue every kernel of one trial on st (the trial's shape is fixed by the
// host-side atom bound, the rebuild interval and N_f; the kernels read
// everything else from the control block).  With timing, HIP events bracket
// each step kernel.
int enqueue_trial(h4d_system *s, int move, hipStream_t st, int nf, int M, bool timing) {
    KArgs &a = s->a;
    const int n_all_max = s->n_host + 2;
    const int G = blocks_for(n_all_max);                 // one thread per atom
    const int GA = atom_blocks_l(n_all_max, a.lanes);    // lanes threads per atom
    int rc;
    hipLaunchKernelGGL(k_propose, dim3(1), dim3(kBlock), 0, st, a, move);
    if ((rc = sort_in(s, n_all_max, st))) return rc;
    hipLaunchKernelGGL(k_energy, dim3(GA), dim3(kBlock), 0, st, a, 0, -1, 0.0, 0);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, st, a, 0, GA);
    int b = 0;
    const bool final_rebuild = nf % M != 0;   // the end energy needs a list without fast atoms
    for (int k = 0; k <= nf; ++k) {
        if (k > 0 && k % M == 0)
            if ((rc = rebuild_mid(s, b, n_all_max, st))) return rc;
        const int bin = !a.G.use_cells ? 0 : ((k + 1) % M == 0 && k + 1 <= nf ? 1 : (k == nf && final_rebuild ? 1 : 0));
        hipEvent_t e0 = timing ? s->ev[2 * k] : nullptr, e1 = timing ? s->ev[2 * k + 1] : nullptr;
        if (s->p.precision == H4D_PREC_FP32) launch_step<1>(s, st, GA + 1, e0, e1, k, b, bin);
        else launch_step<0>(s, st, GA + 1, e0, e1, k, b, bin);
        if (a.G.water)
            hipLaunchKernelGGL(k_settle, dim3(blocks_for(a.G.n_mol)), dim3(kBlock), 0, st, a, k, b, bin, s->cl);
        b ^= 1;
    }
    if (final_rebuild && (rc = rebuild_mid(s, b, n_all_max, st))) return rc;
    s->last_buf = b;
    hipLaunchKernelGGL(k_energy, dim3(GA), dim3(kBlock), 0, st, a, 1, -1, 0.0, b);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, st, a, 1, GA);
    hipLaunchKernelGGL(k_metropolis, dim3(1), dim3(1), 0, st, a);
    hipLaunchKernelGGL(k_commit, dim3(G), dim3(kBlock), 0, st, a, b);
    hipLaunchKernelGGL(k_compact1, dim3(G), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_compact2, dim3(G), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_commit_ctl, dim3(1), dim3(1), 0, st, a);
    HIPC(hipGetLastError());
    return H4D_OK;
}

int launch_trial(h4d_system *s, int move) {
    KArgs &a = s->a;
    hipStream_t st = s->stream;
    const int nf = s->p.n_steps_max > 0 ? s->p.n_steps_max : s->p.n_steps;
    const int M = std::max(1, s->trial_M);
    int rc;
    s->trial_rebuilds = nf / M + (nf % M != 0 ? 1 : 0);
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
        const int n_all_max = s->n_host + 2;
        const auto key = std::make_tuple(blocks_for(n_all_max), atom_blocks_l(n_all_max, a.lanes), M, nf, move, tm,
                                         a.lanes);
        auto it = s->graphs.find(key);
        if (it == s->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            bool ok = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            int erc = ok ? enqueue_trial(s, move, s->cap_stream, nf, M, s->timing) : H4D_OK;
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
    if (!launched && (rc = enqueue_trial(s, move, st, nf, M, s->timing))) return rc;
    HIPC(hipMemcpyAsync(s->h_rec, a.rec, sizeof(TrialRec), hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(s->h_ctl, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (s->timing) {
        const int nf_dev = std::min(s->h_ctl->nf, nf);
        for (int k = 0; k <= nf_dev; ++k) {
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, s->ev[2 * k], s->ev[2 * k + 1]));
            s->step_ms += ms;
            s->step_launches += 1;
        }
    }
    return H4D_OK;
}

int run_one(h4d_system *s, int move, h4d_trial *out) {
    bool retried = false;
    s->trial_M = std::max(1, s->rebuild_every);
    for (int attempt = 0; attempt < 16; ++attempt) {
        int rc = launch_trial(s, move);
        if (rc) return rc;
        const Ctl *c = s->h_ctl;
        if (c->retry) {
            const unsigned err = c->err;
            if (err & kErrCap) return fail(H4D_ECAPACITY, "atom capacity exhausted");
            if ((rc = grow_lists(s, err))) return rc;
            // more fast atoms than the fast list holds: recompute this trial
            // with a shorter rebuild interval, and shorten the base interval
            if (err & (kErrSkin | kErrFast)) {
                s->trial_M = std::max(1, s->trial_M / 2);
                if (s->p.rebuild_every == 0) s->rebuild_every = std::max(1, (s->rebuild_every * 3) / 4);
                s->clean_trials = 0;
            }
            if ((rc = clear_errors(s))) return rc;
            retried = true;
            s->retries += 1;
            continue;
        }
        h4d_trial r;
        std::memcpy(&r, s->h_rec, sizeof(r));
        if (retried) r.flags |= H4D_FLAG_RETRIED;
        r.n_rebuilds = s->trial_rebuilds;
        if (out) *out = r;
        s->n_host = c->n;
        s->nsalt_host = c->nsalt;
        s->n_trials += 1;
        if (r.move > 0) { s->n_ins += 1; s->n_ins_acc += r.accepted; }
        else { s->n_del += 1; s->n_del_acc += r.accepted; }
        // automatic rebuild interval: lengthen it after a run of trials whose
        // fast lists stayed short (a few percent of their capacity)
        if (s->p.rebuild_every == 0 && !retried) {
            if (c->max_fast <= kFastCap / 16) {
                if (++s->clean_trials >= 20) { s->rebuild_every += 1; s->clean_trials = 0; }
            } else {
                s->clean_trials = 0;
            }
        }
        s->N_sum += (double)c->nsalt;
        s->N2_sum += (double)c->nsalt * (double)c->nsalt;
        return H4D_OK;
    }
    return fail(H4D_EHIP, "trial could not be completed after resizing the lists");
}

}  // namespace

extern "C" {

const char *h4d_last_error(void) { return g_err.c_str(); }

int32_t h4d_init_system(const h4d_params *params, int32_t n_atoms, int32_t n_salt, int32_t n_mol,
                        const double *pos, const int32_t *type, const int32_t *mol, const int64_t *tag,
                        void *hip_stream, h4d_system **out) {
    g_err.clear();
    if (!params || !out || n_atoms < 0 || n_salt < 0 || (n_atoms > 0 && (!pos || !type || !tag)))
        return fail(H4D_EINVAL, "null argument or negative size");
    *out = nullptr;
    int rc = check_params(*params);
    if (rc) return rc;
    int ndev = 0;
    const hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev < 1)
        return fail(H4D_ENODEV, std::string("no HIP device (hipGetDeviceCount: ") + hipGetErrorString(de) +
                                    ", count " + std::to_string(ndev) + ")");
    // validate the configuration
    int ncat = 0, nan_ = 0;
    for (int i = 0; i < n_atoms; ++i) {
        if (type[i] < 0 || type[i] >= params->n_types) return fail(H4D_EINVAL, "atom type out of range");
        ncat += type[i] == params->cation_type;
        nan_ += type[i] == params->anion_type;
        if (i > 0 && tag[i] <= tag[i - 1]) return fail(H4D_EINVAL, "tags must ascend in array order");
        for (int d = 0; d < 3; ++d)
            if (!(pos[3 * i + d] >= 0.0 && pos[3 * i + d] < params->box[d]))
                return fail(H4D_EINVAL, "positions must lie in [0, L)");
    }
    if (ncat != n_salt || nan_ != n_salt) return fail(H4D_EINVAL, "n_salt must equal the cation and anion counts");
    if (params->water) {
        if (n_mol < 1 || 3 * n_mol > n_atoms || !mol) return fail(H4D_EINVAL, "water = 1 needs n_mol >= 1 waters first");
        for (int m = 0; m < n_mol; ++m)
            for (int q = 0; q < 3; ++q) {
                const int i = 3 * m + q;
                if (mol[i] != m || type[i] != type[q]) return fail(H4D_EINVAL, "waters must be atoms 3m, 3m+1, 3m+2 (O, H, H) of molecule m");
            }
        if (type[1] != type[2] || type[0] == type[1]) return fail(H4D_EINVAL, "water atoms must be O, H, H");
        for (int i = 3 * n_mol; i < n_atoms; ++i)
            if (mol[i] >= 0) return fail(H4D_EINVAL, "only the waters may carry molecule ids");
    } else if (mol) {
        for (int i = 0; i < n_atoms; ++i)
            if (mol[i] >= 0) return fail(H4D_EINVAL, "molecule ids need water = 1");
    }

    auto *s = new h4d_system();
    s->p = *params;
    if (const char *e = std::getenv("H4D_NO_GRAPHS")) {
        if (e[0] == '1') s->graphs_ok[0] = false;   // launch every kernel eagerly
    }
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->cap = params->capacity > 0 ? params->capacity : n_atoms + 4096;
    if (s->cap < n_atoms + 2) { delete s; return fail(H4D_EINVAL, "capacity below n_atoms + 2"); }
    s->n_host = n_atoms;
    s->nsalt_host = n_salt;
    s->n_mol = n_mol;
    setup_geo(s);
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
    if (!s->a.G.use_cells && s->cap > 8192) {
        delete s;
        return fail(H4D_EINVAL, "a box with fewer than 3 list cells per edge is limited to 8192 atoms");
    }
    {
        int L = params->lanes_per_atom;
        if (L == 0) L = n_atoms <= 16384 ? 16 : (n_atoms <= 65536 ? 8 : 4);
        s->a.lanes = L;
        s->a.lanes_log2 = L == 4 ? 2 : (L == 8 ? 3 : 4);
    }
    initial_capacities(s, n_atoms);
    KArgs &a = s->a;
    a.cap = s->cap;
    a.seed = params->seed;
    a.stream = params->stream;
    a.n_steps = params->n_steps;
    a.n_steps_min = params->n_steps_min;
    a.n_steps_max = params->n_steps_max;
    a.cation_type = params->cation_type;
    a.anion_type = params->anion_type;
    s->partial_blocks = atom_blocks_l(s->cap + 2, kMaxLanes) + 1;   // every energy grid fits
    const size_t C = (size_t)s->cap;
    PairCoef *coef_d = nullptr;
    double *mass_d = nullptr;
    if ((rc = s->alloc(&a.cpos, C)) || (rc = s->alloc(&a.ctag, C)) || (rc = s->alloc(&a.ctype, C)) ||
        (rc = s->alloc(&a.cmol, C)) || (rc = s->alloc(&a.pos[0], C)) || (rc = s->alloc(&a.pos[1], C)) ||
        (rc = s->alloc(&a.fx[0], C)) || (rc = s->alloc(&a.fx[1], C)) || (rc = s->alloc(&a.vel[0], C)) ||
        (rc = s->alloc(&a.vel[1], C)) || (rc = s->alloc(&a.perm, C)) || (rc = s->alloc(&a.wmol, C)) ||
        (rc = s->alloc(&a.posb, C)) || (rc = s->alloc(&a.force, C)) || (rc = s->alloc(&a.tpos, C)) ||
        (rc = s->alloc(&a.ttag, C)) || (rc = s->alloc(&a.ttype, C)) || (rc = s->alloc(&a.tmol, C)) ||
        (rc = s->alloc(&a.nnbr, C)) || (rc = s->alloc(&a.partial, (size_t)s->partial_blocks * 5)) ||
        (rc = s->alloc(&a.ctl, 1)) || (rc = s->alloc(&a.rec, 1)) ||
        (rc = s->alloc(&a.molw, (size_t)std::max(1, 3 * n_mol))) || (rc = s->alloc(&a.fw, C)) ||
        (rc = s->alloc(&coef_d, (size_t)kMaxTypes * kMaxTypes)) || (rc = s->alloc(&mass_d, kMaxTypes)) ||
        (rc = alloc_lists(s))) {
        delete s;
        return rc;
    }
    a.coef = coef_d;
    a.mass = mass_d;
    if (hipHostMalloc((void **)&s->h_rec, sizeof(TrialRec)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_ctl, sizeof(Ctl)) != hipSuccess) {
        delete s;
        return fail(H4D_ENOMEM, "pinned host allocation failed");
    }
    // upload
    std::vector<double4> hp(std::max(1, n_atoms));
    std::vector<int> hm(std::max(1, n_atoms), -1);
    for (int i = 0; i < n_atoms; ++i) {
        long long meta = type[i];
        double wbits;
        std::memcpy(&wbits, &meta, sizeof(wbits));
        hp[i] = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], wbits);
        if (mol) hm[i] = mol[i];
    }
    std::memset(s->h_ctl, 0, sizeof(Ctl));
    Ctl &c = *s->h_ctl;
    c.n = n_atoms;
    c.n_all = n_atoms;
    c.nsalt = n_salt;
    c.next_tag = n_atoms ? tag[n_atoms - 1] + 1 : 0;
    c.trial = 0;
    c.nf = 0;
    c.ic = c.ia = -1;
    double mass_h[kMaxTypes] = {0};
    for (int t = 0; t < params->n_types; ++t) mass_h[t] = params->mass[t];
#define UPLOAD(dst, src, bytes)                                                                        \
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {                           \
        delete s;                                                                                      \
        return fail(H4D_EHIP, "upload failed");                                                       \
    }
    if (n_atoms > 0) {
        UPLOAD(a.cpos, hp.data(), sizeof(double4) * n_atoms);
        UPLOAD(a.ctype, type, sizeof(int) * n_atoms);
        UPLOAD(a.cmol, hm.data(), sizeof(int) * n_atoms);
        UPLOAD(a.ctag, tag, sizeof(long long) * n_atoms);
    }
    UPLOAD(a.ctl, &c, sizeof(Ctl));
    UPLOAD(coef_d, s->coef_h, sizeof(s->coef_h));
    UPLOAD(mass_d, mass_h, sizeof(mass_h));
#undef UPLOAD
    // rebuild interval: the fastest atoms (5 standard deviations) cover half
    // the skin; adapted on overflow
    double m_min = params->mass[0];
    for (int t = 1; t < params->n_types; ++t) m_min = std::min(m_min, params->mass[t]);
    const double vmax = 5.0 * std::sqrt(params->accel * params->kT / m_min);
    s->rebuild_every = params->rebuild_every > 0
                           ? params->rebuild_every
                           : std::max(1, (int)std::floor(0.5 * params->skin / (vmax * params->dt)));
    if ((rc = h4d_build_neighbors(s))) { delete s; return rc; }
    *out = s;
    return H4D_OK;
}

int32_t h4d_build_neighbors(h4d_system *s) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    for (int attempt = 0; attempt < 8; ++attempt) {
        int rc = sort_in(s, s->n_host, s->stream);
        if (rc) return rc;
        if ((rc = read_ctl(s))) return rc;
        const unsigned err = s->h_ctl->err;
        if (!(err & (kErrNbr | kErrCell))) return H4D_OK;
        if ((rc = grow_lists(s, err))) return rc;
        if ((rc = clear_errors(s))) return rc;
    }
    return fail(H4D_ECAPACITY, "neighbour lists could not be sized");
}

int32_t h4d_run_nemd_trial(h4d_system *s, int32_t move, h4d_trial *out) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    return run_one(s, move, out);
}

int32_t h4d_run_trials(h4d_system *s, int32_t n, int32_t move, h4d_trial *out) {
    if (!s || n < 0) return fail(H4D_EINVAL, "null handle or negative count");
    if (move < -1 || move > 1) return fail(H4D_EINVAL, "move must be -1, 0 or +1");
    for (int q = 0; q < n; ++q) {
        int rc = run_one(s, move, out ? out + q : nullptr);
        if (rc) return rc;
    }
    return H4D_OK;
}

int32_t h4d_set_trial_index(h4d_system *s, uint64_t trial) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    int rc = read_ctl(s);
    if (rc) return rc;
    s->h_ctl->trial = (long long)trial;
    HIPC(hipMemcpyAsync(s->a.ctl, s->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int32_t h4d_get_state(h4d_system *s, int32_t cap, int32_t *n, int32_t *n_salt, double *pos, double *vel,
                      int32_t *type, int32_t *mol, int64_t *tag) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    int rc = read_ctl(s);
    if (rc) return rc;
    const int nn = s->h_ctl->n;
    if (n) *n = nn;
    if (n_salt) *n_salt = s->h_ctl->nsalt;
    if ((pos || vel || type || mol || tag) && cap < nn) return fail(H4D_EINVAL, "cap smaller than the atom count");
    std::vector<double4> buf(std::max(1, nn));
    if (pos && nn) {
        HIPC(hipMemcpy(buf.data(), s->a.cpos, sizeof(double4) * nn, hipMemcpyDeviceToHost));
        for (int i = 0; i < nn; ++i) { pos[3 * i] = buf[i].x; pos[3 * i + 1] = buf[i].y; pos[3 * i + 2] = buf[i].z; }
    }
    if (vel && nn) {
        // velocities are those of the last trajectory's end, in canonical order
        std::vector<int> perm(nn);
        HIPC(hipMemcpy(perm.data(), s->a.perm, sizeof(int) * nn, hipMemcpyDeviceToHost));
        HIPC(hipMemcpy(buf.data(), s->a.vel[s->last_buf], sizeof(double4) * nn, hipMemcpyDeviceToHost));
        for (int w = 0; w < nn; ++w) {
            const int i = perm[w];
            if (i < 0 || i >= nn) continue;
            vel[3 * i] = buf[w].x; vel[3 * i + 1] = buf[w].y; vel[3 * i + 2] = buf[w].z;
        }
    }
    if (type && nn) HIPC(hipMemcpy(type, s->a.ctype, sizeof(int) * nn, hipMemcpyDeviceToHost));
    if (mol && nn) HIPC(hipMemcpy(mol, s->a.cmol, sizeof(int) * nn, hipMemcpyDeviceToHost));
    if (tag && nn) HIPC(hipMemcpy(tag, s->a.ctag, sizeof(long long) * nn, hipMemcpyDeviceToHost));
    return H4D_OK;
}

}  // extern "C"

namespace {

// FP64 energies of the working buffer-0 state (after sort_in).
int energies(h4d_system *s, int mode, double w, double out[4]) {
    KArgs &a = s->a;
    const int GA = atom_blocks_l(s->n_host, a.lanes);
    hipLaunchKernelGGL(k_energy, dim3(GA), dim3(kBlock), 0, s->stream, a, 2, mode, w, 0);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s->stream, a, 2, GA);
    HIPC(hipGetLastError());
    int rc = read_ctl(s);
    if (rc) return rc;
    out[0] = s->h_ctl->Ulj + s->h_ctl->Uc;
    out[1] = s->h_ctl->Ulj;
    out[2] = s->h_ctl->Uc;
    out[3] = s->h_ctl->vir;
    return H4D_OK;
}

}  // namespace

extern "C" {

int32_t h4d_forces_at(h4d_system *s, const int32_t flying[2], double w, double *forces, double *energy) {
    if (!s || !flying) return fail(H4D_EINVAL, "null argument");
    const int n = s->n_host;
    for (int q = 0; q < 2; ++q)
        if (flying[q] < -1 || flying[q] >= n) return fail(H4D_EINVAL, "flying index out of range");
    KArgs &a = s->a;
    for (int q = 0; q < 2; ++q)
        if (flying[q] >= 0) hipLaunchKernelGGL(k_set_fly, dim3(1), dim3(1), 0, s->stream, a, flying[q], 1);
    int rc = h4d_build_neighbors(s);
    if (rc) return rc;
    if (s->p.precision == H4D_PREC_FP32) launch_forces<1>(s, atom_blocks_l(n, a.lanes), w);
    else launch_forces<0>(s, atom_blocks_l(n, a.lanes), w);
    HIPC(hipGetLastError());
    double e[4];
    if ((rc = energies(s, 0, w, e))) return rc;
    if (forces && n) {
        std::vector<double4> buf(n);
        HIPC(hipMemcpy(buf.data(), a.force, sizeof(double4) * n, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) {
            forces[3 * i] = buf[i].x;
            forces[3 * i + 1] = buf[i].y;
            forces[3 * i + 2] = buf[i].z;
        }
    }
    if (energy) { energy[0] = e[0]; energy[1] = e[1]; energy[2] = e[2]; }
    for (int q = 0; q < 2; ++q)
        if (flying[q] >= 0) hipLaunchKernelGGL(k_set_fly, dim3(1), dim3(1), 0, s->stream, a, flying[q], 0);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s->stream));
    return H4D_OK;
}

int32_t h4d_sample_observables(h4d_system *s, h4d_observables *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    double e[4];
    int rc = h4d_build_neighbors(s);
    if (rc) return rc;
    if ((rc = energies(s, 0, 0.0, e))) return rc;
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    const Ctl *c = s->h_ctl;
    out->n_atoms = c->n;
    out->n_salt = c->nsalt;
    out->n_trials = s->n_trials;
    out->n_ins = s->n_ins;
    out->n_ins_acc = s->n_ins_acc;
    out->n_del = s->n_del;
    out->n_del_acc = s->n_del_acc;
    out->U = e[0];
    out->U_lj = e[1];
    out->U_coul = e[2];
    out->virial = e[3];
    out->pressure_virial = ((double)c->n * s->p.kT + e[3] / 3.0) / s->a.G.volume;
    if (s->n_trials > 0) {
        out->N_mean = s->N_sum / (double)s->n_trials;
        out->N2_mean = s->N2_sum / (double)s->n_trials;
        out->chi = out->N_mean > 0.0 ? (out->N2_mean - out->N_mean * out->N_mean) / out->N_mean : 0.0;
    }
    return H4D_OK;
}

int32_t h4d_set_timing(h4d_system *s, int32_t on) {
    if (!s) return fail(H4D_EINVAL, "null handle");
    if ((on != 0) != s->timing) s->drop_graphs();
    s->timing = on != 0;
    s->retries = 0;
    s->step_launches = 0;
    s->step_ms = 0.0;
    return H4D_OK;
}

int32_t h4d_get_timing(h4d_system *s, h4d_timing *out) {
    if (!s || !out) return fail(H4D_EINVAL, "null argument");
    unsigned long long *d = nullptr;
    int rc = s->alloc(&d, 1);
    if (rc) return rc;
    HIPC(hipMemsetAsync(d, 0, sizeof(*d), s->stream));
    hipLaunchKernelGGL(k_sum_nbr, dim3(blocks_for(s->n_host)), dim3(kBlock), 0, s->stream, s->a, d);
    unsigned long long sum = 0;
    HIPC(hipMemcpyAsync(&sum, d, sizeof(sum), hipMemcpyDeviceToHost, s->stream));
    HIPC(hipStreamSynchronize(s->stream));
    s->release(d);
    out->step_launches = s->step_launches;
    out->step_ms = s->step_ms;
    out->mean_nbr = s->n_host > 0 ? (double)sum / (double)s->n_host : 0.0;
    out->rebuild_every = s->rebuild_every;
    out->nbr_cap = s->a.nbr_cap;
    out->lanes = s->a.lanes;
    out->cell_cap = s->a.cell_cap;
    out->retries = s->retries;
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
