#!/usr/bin/env python3
"""Throughput of H4D salt-pair exchange trials on one MI355X, learned vs plain.

Default workload (N = 1), the aqueous NaCl box with the learned proposal:
8,000 rigid SPC/E waters + 150 Na+/Cl- pairs in a 62 A box at 298 K; every
trial flies one NaCl pair in or out along w in 500 velocity-Verlet steps of
1 fs (w_max 3 A, kappa_sr 1/A, DSF Coulomb alpha 0.25/A cut 10 A); FP32 pair
arithmetic on FP64 positions, velocities, energies, work and Metropolis
ratio.  Two arms run the same chain from the same start state, each on 8
speculative replicas of the box (a batch of replica boxes in one engine, the
chain's records equal to a one-by-one run):
  plain    the uniform pair insertion of Eq. (4);
  learned  the multiple-try proposal over 4,096 uniform candidate sites per
           attempt (Sec. II B 4, Eqs. 15-16, with a learned weight), each
           scored by the network (64 features -> 3 x 128 GELU -> 1) in BF16
           on the matrix cores, the ratio corrected exactly.
Before the timed region: the lattice start relaxes through equilibrium
phases (generalized hybrid MC); pilot insertions and deletions on that state
(forced moves that are never accepted, so the state stays fixed) give the
operating beta mu by Bennett's acceptance ratio (Crooks' relation, the
supplement's CFT/BAR section) and the network's training data (features and
work of the method's own moves); the network trains on the GPU (FP32
forward, backward, Adam); a fixed-state comparison of a few weight scales
picks one, and a second one on fresh trials compares it with the uniform
proposal (expected acceptance in log space: at the equilibrium beta mu of
0.5 ps flights it underflows).

One "step" of this benchmark is one exchange trial of the chain.  value =
NEMD atom-steps/s of the learned arm (the whole hot path, candidate scoring
included); the plain arm, accepted exchanges/s of both arms with Wilson
intervals, and the fixed-state comparison stand beside it.  Extra keys: the
32,000-ion LJ chain with the same learned-vs-plain study (there exchanges
are frequent enough to count), and the 256-box batch (--no-extras leaves
them out).

Other workloads: --workload lj32k (32,000 LJ ions), --workload batched (256
independent LJ boxes of 1,000-16,000 ions).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted salt-pair exchanges/s + NEMD atom-steps/s (1 GPU), learned vs plain"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # published vector FP32 rate (packed FP32 counted)
# committed counter summaries of the step kernel, one per workload, lanes per
# atom and list-load kind (the autotuner's choices decide which instantiation
# the bench times; each file names the ones it was taken with)
TRAFFIC_FILES = {
    "water": [os.path.join(ROOT, "profiles", "k_step_water_traffic.txt"),
              os.path.join(ROOT, "profiles", "k_step_water_l8_traffic.txt")],
    "lj32k": [os.path.join(ROOT, "profiles", "k_step_lj32k_traffic.txt")],
    "batched": [os.path.join(ROOT, "profiles", "k_step_batched256_traffic.txt")],
}
COUNTER_FILES = {
    "water": [os.path.join(ROOT, "profiles", "k_step_water_counters.txt"),
              os.path.join(ROOT, "profiles", "k_step_water_l8_counters.txt")],
}


def _summary_fields(path):
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    return kv


def _matching_summary(files, lanes, nt):
    """The committed summary taken on the current kernel sources with these
    lanes per atom and list-load kind, or None."""
    from paper_2307_11447_amd import rocprof_summary
    for path in files:
        if not os.path.exists(path):
            continue
        kv = _summary_fields(path)
        if (kv.get("kernel_source_sha256") == rocprof_summary.kernel_source_hash() and
                kv.get("lanes_per_atom") == str(lanes) and kv.get("nontemporal_lists") == str(nt)):
            return path
    return None
CANDIDATES = 4096
INSERT_SHIFTS = (0, 20, 40, 60, 80, 100, 120)   # beta mu above the operating point, insertion curves


def note(msg):
    """Progress of the run on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def wilson(k, n, z=1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def host_cores():
    """Threads of the CPU baseline: OMP_NUM_THREADS if set, else the
    process's CPUs, at most 16 (the host share of one GPU)."""
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if env > 0:
        return env
    return max(1, min(16, len(os.sched_getaffinity(0))))


# ---------------------------------------------------------------------------
# Roofline of the fused step kernel
# ---------------------------------------------------------------------------
def step_bytes_per_atom(mean_nbr):
    """Algorithmic HBM bytes of one atom-step of the fused step kernel: the
    pair pass, 4 B per list entry + 16 B own coordinates, charge and type +
    16 B force + 4 B list length (4 n_list + 36), plus the velocity-Verlet
    update, 120 B (FP64 position and velocity in and out, FP32 force);
    neighbour records are gathered through the caches and not counted."""
    return 4.0 * mean_nbr + 36.0 + 120.0


def step_flop_per_atom(mean_nbr):
    """Floating-point operations of one atom-step (an FMA counts 2, a
    reciprocal, square root or exponential 1): per list entry, in FP32, the
    displacement and squared 4D distance (9), the LJ force factor with 1/s^2
    (7), the DSF Coulomb force factor with s, 1/s, the Gaussian and the erfc
    approximation (23), their sum (1) and the accumulation (6): 46; per atom,
    in FP64, the two half kicks and the drift (18)."""
    return 46.0 * mean_nbr + 18.0


def counted_traffic(workload, timing):
    """HBM bytes per step launch from the committed rocprofv3 counter summary
    of this workload's step kernel in the instantiation the timing describes
    (lanes per atom, list-load kind), or None if there is none or it was
    taken on different kernel sources."""
    path = _matching_summary(TRAFFIC_FILES.get(workload, []), timing["lanes"], timing["nt_lists"])
    if path is None:
        return None
    try:
        return float(_summary_fields(path)["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counted_valu_busy(workload, timing):
    """rocprofv3's VALUBusy (percent) of the step kernel in the instantiation
    the timing describes, from the committed counter summary, or None."""
    path = _matching_summary(COUNTER_FILES.get(workload, []), timing["lanes"], timing["nt_lists"])
    if path is None:
        return None
    kernel_substr = f"k_step<1, {timing['lanes']}, false, {'true' if timing['nt_lists'] else 'false'}>"
    for line in open(path):
        if kernel_substr in line and " VALUBusy " in line and "mean=" in line:
            return float(line.rsplit("mean=", 1)[1])
    return None


def roofline(timing, traffic_bytes, kernel, valu_busy=None):
    """The step kernel against the HBM roofline: algorithmic bytes of the
    atoms its timed launches integrated over their summed HIP-event time."""
    n_l = timing["mean_nbr"]
    step_s = max(timing["step_ms"], 1e-300) * 1e-3
    launches = max(1, timing["step_launches"])
    atoms = timing["atom_launches"]
    bpa, fpa = step_bytes_per_atom(n_l), step_flop_per_atom(n_l)
    achieved = bpa * atoms / step_s / 1e9
    flops = fpa * atoms / step_s / 1e12
    return {
        "kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": None if traffic_bytes is None else traffic_bytes * launches / step_s / 1e9,
        "traffic_bytes_per_launch": traffic_bytes,
        "valu_busy_pct": valu_busy,
        "bytes_per_atom_step": bpa, "mean_list_entries": n_l,
        "atom_launches": atoms, "launches": timing["step_launches"],
        "avg_kernel_us": 1e3 * timing["step_ms"] / launches,
        "flop": {"achieved": flops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": flops / FP32_VECTOR_PEAK_TFLOPS, "flop_per_atom_step": fpa},
        "timing": "HIP events around every step-kernel launch of the timing trials, on the library's stream",
    }


# ---------------------------------------------------------------------------
# CPU baseline: the oracle's OpenMP timing build in a child process
# ---------------------------------------------------------------------------
def _oracle_trial(args):
    root, threads, params, x, type_, mol, tag, nsalt, n_mol, t, move = args
    os.environ["OMP_NUM_THREADS"] = str(threads)
    if root not in sys.path:
        sys.path.insert(0, root)
    from oracle import oracle as O
    O.use_timing_build()
    o = O.OracleSystem(params, x, type_, mol, tag, nsalt, n_mol=n_mol, cap=len(type_) + 8)
    t0 = time.perf_counter()
    rec = o.trial(t, move)
    return time.perf_counter() - t0, rec["move"], rec["n_steps"]


def cpu_baseline(w, n_steps, label, beta_mu):
    """The FP64 oracle (its OpenMP timing build, on the host's cores) on one
    trial of the workload's start state with N_f = n_steps."""
    cores = host_cores()
    params = dict(w.params, n_steps=n_steps, n_steps_min=0, n_steps_max=0, beta_mu=beta_mu)
    job = (ROOT, cores, params, w.x, w.type, w.mol, w.tag, w.nsalt, w.n_mol, 0, 1)
    with mp.get_context("spawn").Pool(1) as pool:
        dt, move, nf = pool.apply(_oracle_trial, (job,))
    atom_steps = w.n * nf
    return {"value": atom_steps / dt, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"1 insertion trial of {label} with N_f = {nf} ({atom_steps:.3g} atom-steps, {dt:.1f} s), "
                      f"OpenMP build of the oracle on {cores} threads",
            "trials_per_s": 1.0 / dt}


# ---------------------------------------------------------------------------
# Acceptance statistics of trial records
# ---------------------------------------------------------------------------
def expected_acceptance(recs, move=0):
    """Mean Metropolis acceptance min(1, exp(ln R)) of the records (of one
    kind of move if given): an estimator of the acceptance rate with far less
    variance than the count of accepted trials when acceptance is rare."""
    vals = []
    for r in recs:
        if move and r.move != move:
            continue
        lr = r.ln_ratio
        vals.append(0.0 if (r.flags & 0x3) or not math.isfinite(lr) else math.exp(min(0.0, lr)))
    return sum(vals) / max(1, len(vals)), len(vals)


def arm_summary(recs, wall, rounds=None):
    n = len(recs)
    atom_steps = sum(r.n_atoms * r.n_steps for r in recs)
    acc = sum(r.accepted for r in recs)
    ins = [r for r in recs if r.move > 0]
    dels = [r for r in recs if r.move < 0]
    lo, hi = wilson(acc, n)
    e_all, _ = expected_acceptance(recs)
    e_ins, n_ins = expected_acceptance(recs, 1)
    e_del, n_del = expected_acceptance(recs, -1)
    ns = [r.n_salt_after for r in recs]
    out = {
        "atom_steps_per_s": atom_steps / wall, "trials": n, "wall_s": wall, "trials_per_s": n / wall,
        "accepted": acc, "accepted_exchanges_per_s": acc / wall,
        "p_acc": acc / max(1, n), "p_acc_wilson95": [lo, hi],
        "insertions": n_ins, "insertions_accepted": sum(r.accepted for r in ins),
        "deletions": n_del, "deletions_accepted": sum(r.accepted for r in dels),
        "p_ins_wilson95": list(wilson(sum(r.accepted for r in ins), len(ins))),
        "p_del_wilson95": list(wilson(sum(r.accepted for r in dels), len(dels))),
        "expected_p_ins": e_ins, "expected_p_del": e_del,
        "expected_exchanges_per_s": e_all * n / wall,
        "n_salt_first": recs[0].n_salt_before if recs else None, "n_salt_last": ns[-1] if ns else None,
        "n_salt_mean": sum(ns) / max(1, len(ns)),
        "retried_trials": sum(1 for r in recs if r.flags & 0x4),
        "nonfinite_trials": sum(1 for r in recs if r.flags & 0x2),
    }
    if rounds is not None:
        out["rounds"] = rounds
    return out


def timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def relaxed(h4d, w, phases, steps):
    """The workload's start state after `phases` equilibrium phases of
    `steps` steps (generalized hybrid MC with a full momentum refresh: each
    phase starts from fresh Maxwell-Boltzmann momenta, so the excess energy
    of the lattice start leaves with the old ones), as a workload."""
    import dataclasses
    g = h4d.System.from_workload(w, md_refresh=0.0)
    acc = sum(g.md_phase(steps)[0]["accepted"] for _ in range(phases))
    st = g.state()
    g.close()
    note(f"relaxation: {phases} phases of {steps} steps, {acc} accepted")
    return dataclasses.replace(w, x=st["x"], type=st["type"], mol=st["mol"], tag=st["tag"], nsalt=int(st["nsalt"]))


# ---------------------------------------------------------------------------
# Pilot, chemical potential, network and its weighting
# ---------------------------------------------------------------------------
def pilot(sys_, h4d, n_ins, n_del):
    """Forced uniform insertions (beta mu = -1000) and deletions (+1000) on
    the handle's state: never accepted, so the state stays fixed.  Returns
    the records and each moved site's 64 features."""
    sys_.set_proposal(None, 1)          # equal weights, k = 1: uniform, features recorded
    out = {}
    for key, move, bm, n in (("ins", h4d.MOVE_INSERT, -1.0e3, n_ins), ("del", h4d.MOVE_DELETE, 1.0e3, n_del)):
        sys_.set_beta_mu(bm)
        recs, feats = [], []
        for _ in range(n):
            recs.append(sys_.trial(move))
            feats.append(sys_.last_site_features())
        out[key] = (recs, feats, bm)
    sys_.set_proposal(None, 0)
    return out


def train_network(h4d, X, y, epochs, seed=1):
    """The proposal network trained on the GPU (FP32 forward, backward and
    Adam with decoupled weight decay; batch 128, lr 1e-3)."""
    net = h4d.Mlp(seed=seed)
    steps = max(50, (epochs * len(X)) // 128)
    losses = net.train(X, y, steps=steps, batch=128, lr=1e-3, seed=seed + 1, weight_decay=1e-2)
    return net, steps, losses


def out_of_fold(h4d, X, y, epochs, folds=5):
    """Logits of every pilot site from a network trained without it."""
    import numpy as np
    oof = np.zeros(len(X))
    fold = np.arange(len(X)) % folds
    for f in range(folds):
        tr, te = fold != f, fold == f
        net, _, _ = train_network(h4d, X[tr], y[tr], epochs, seed=10 + f)
        oof[te] = net.forward(X[te])
        net.close()
    return oof


def finite_json(x):
    """x with every non-finite float replaced by None (strict JSON)."""
    if isinstance(x, dict):
        return {k: finite_json(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite_json(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def log_mean_exp(v):
    """ln of the mean of exp(v) (entries of -inf count as zeros)."""
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    if len(v) == 0 or not np.isfinite(v.max()):
        return -math.inf
    m = v.max()
    return float(m + math.log(np.exp(v - m).sum()) - math.log(len(v)))


def proposal_ab(sys_, torch, h4d, arms, beta_mu, n_each, block=50):
    """Insertion and deletion acceptance of several proposals on one fixed
    state: forced moves at beta mu = -1000 (insertions) and +1000
    (deletions), which are never accepted, so the state does not change;
    each record's ln R is moved to the operating beta mu and the mean of
    min(1, R) taken -- in log space, since at an equilibrium beta mu with
    short flights it underflows.  The arms alternate in blocks so that they
    share the same state and device conditions.  arms: name -> (net, k,
    scale, cap[, (x_b, alpha_b, v_ex_edge)]) (k = 0: the uniform proposal;
    the optional last entry sets the bimodal bias and early rejection)."""
    import numpy as np
    out = {name: {"ins": [], "del": [], "ins_ln_r": [], "del_ln_r": [], "s": 0.0, "n": 0, "instant": 0}
           for name in arms}
    done = 0
    while done < n_each:
        nb = min(block, n_each - done)
        for name, spec in arms.items():
            net, k, scale, cap = spec[:4]
            x_b, alpha_b, v_ex = spec[4] if len(spec) > 4 else (0.0, 0.0, 0.0)
            sys_.set_early_rejection(0.0)
            if k > 0:
                sys_.set_bias(0.0, 0.0)
                sys_.set_proposal(net, k, cap, scale)
            else:
                sys_.set_proposal(None, 0)
                sys_.set_bias(x_b, alpha_b)
                sys_.set_early_rejection(v_ex)
            for move, bm, key in ((h4d.MOVE_INSERT, -1.0e3, "ins"), (h4d.MOVE_DELETE, 1.0e3, "del")):
                sys_.set_beta_mu(bm)
                arr, dt = timed(torch, lambda: sys_.trials(nb, move, as_array=True))
                out[name]["s"] += dt
                out[name]["n"] += nb
                shift = (beta_mu - bm) * (1.0 if move > 0 else -1.0)
                for q in range(nb):
                    r = arr[q]
                    ok = not (r.flags & 0x3) and math.isfinite(r.ln_ratio)
                    out[name][key].append(min(0.0, r.ln_ratio + shift) if ok else -math.inf)
                    out[name][key + "_ln_r"].append(r.ln_ratio + shift if ok else -math.inf)
                    out[name]["instant"] += int(bool(r.flags & 0x10))
        done += nb
    sys_.set_proposal(None, 0)
    sys_.set_bias(0.0, 0.0)
    sys_.set_early_rejection(0.0)
    sys_.set_beta_mu(beta_mu)
    res = {}
    ln10 = math.log(10.0)
    for name, o in out.items():
        li, ld = log_mean_exp(o["ins"]), log_mean_exp(o["del"])
        rate = o["n"] / max(1e-300, o["s"])
        lx = math.log(0.5) + np.logaddexp(li, ld) + math.log(rate)
        fi = np.array([v for v in o["ins"] if v > -math.inf])
        fd = np.array([v for v in o["del"] if v > -math.inf])
        res[name] = {"log10_p_insert": li / ln10, "log10_p_delete": ld / ln10,
                     "p_insert": math.exp(li), "p_delete": math.exp(ld), "trials_per_s": rate,
                     "log10_expected_exchanges_per_s": float(lx / ln10), "expected_exchanges_per_s": float(math.exp(lx)),
                     "ln_acc_insert_median": float(np.median(fi)) if len(fi) else None,
                     "ln_acc_delete_median": float(np.median(fd)) if len(fd) else None,
                     "insertions": len(o["ins"]), "deletions": len(o["del"]),
                     "instant_fraction": o["instant"] / max(1, o["n"]),
                     # insertion acceptance as beta mu rises above the operating
                     # point (each ln R moves by the shift): where the uniform
                     # arm accepts insertions at all, the arms compare on many
                     # values instead of a few extreme ones
                     "log10_p_insert_at_beta_mu_plus": {
                         str(sh): log_mean_exp(np.minimum(0.0, np.array(o["ins_ln_r"]) + sh)) / ln10
                         for sh in INSERT_SHIFTS}}
    names = list(arms)
    for other in names[1:]:
        g, ci = ab_log_gain(out[names[0]], out[other])
        res[f"log10_gain_{other}"], res[f"log10_gain_{other}_bootstrap90"] = g, ci
    return res


def ab_log_gain(u, l, reps=1000, seed=11):
    """log10 of the ratio of expected exchanges per second (another proposal
    over the first) and its 90 % bootstrap interval (moves resampled within
    each arm and kind); None where an arm accepts nothing at all."""
    import numpy as np
    rng = np.random.default_rng(seed)

    def lex(o, pick):
        return np.logaddexp(log_mean_exp(pick(o["ins"])), log_mean_exp(pick(o["del"]))) + math.log(o["n"] / o["s"])

    def ident(x):
        return np.asarray(x)

    def res(x):
        x = np.asarray(x)
        return x[rng.integers(0, len(x), len(x))]

    a, b = lex(u, ident), lex(l, ident)
    if not (np.isfinite(a) and np.isfinite(b)):
        return None, None
    boot = []
    for _ in range(reps):
        d = lex(l, res) - lex(u, res)
        if np.isfinite(d):
            boot.append(d)
    ln10 = math.log(10.0)
    lo, hi = np.percentile(boot, [5, 95]) if boot else (math.nan, math.nan)
    return float((b - a) / ln10), [float(lo / ln10), float(hi / ln10)]


def learned_study(args, h4d, torch, w, label, n_ins, n_del, n_select, n_ab, candidates, beta_mu=None):
    """The learned proposal on one state: pilot moves (forced, never
    accepted), beta mu from BAR over them (unless given), the network
    trained on the GPU on the pilot insertions, its weight scale chosen by
    a fixed-state comparison of a few scales, and the final fixed-state
    comparison against the uniform proposal on fresh trials.

    Target: the insertion work itself, -beta dH, centred on its pilot mean
    and clipped to 8 standard deviations.  The multiple-try step depends on
    the log weights only up to a common shift, so the network needs no
    beta mu; the cap on a logit is the largest training target, so the
    choice is never steered beyond what the pilot saw."""
    import numpy as np
    from paper_2307_11447_amd import analysis
    beta = 1.0 / w.params["kT"]
    one = h4d.System.from_workload(w)
    tuned = one.autotune(args.autotune_trials) if args.autotune else None
    if tuned:
        note(f"{label}: autotune: {tuned[0]} lanes per atom, rebuild every {tuned[1]} steps")
    # the tuned lane width; the rebuild interval stays automatic (it adapts to
    # the trials' fast atoms, where a fixed one would recompute every trial
    # whose fast list overflows)
    over = {} if not tuned else dict(lanes_per_atom=tuned[0])
    if args.lanes:
        over["lanes_per_atom"] = args.lanes
    t0 = time.perf_counter()
    pil = pilot(one, h4d, n_ins, n_del)
    pilot_s = time.perf_counter() - t0
    ins_recs, ins_feat, _ = pil["ins"]
    del_recs, _, _ = pil["del"]
    note(f"{label}: pilot: {n_ins} insertions and {n_del} deletions in {pilot_s:.1f} s")
    dM_ins = [r["dM"] for r in ins_recs if not r["flags"] & 0x3]
    dM_del = [r["dM"] for r in del_recs if not r["flags"] & 0x3]
    cal = analysis.work_summary(dM_ins, dM_del, beta, 0.0)
    bmu = beta_mu if beta_mu is not None else cal["beta_mu_bar"]
    cal = analysis.work_summary(dM_ins, dM_del, beta, bmu)
    cal["beta_mu_operating"] = bmu
    cal["note"] = ("uniform forced insertions and deletions on the state (none accepted): beta mu from Bennett's "
                   "acceptance ratio, P_acc predicted by Eq. (21) at the operating beta mu")
    note(f"{label}: BAR beta mu = {cal['beta_mu_bar']:.3f} {cal['beta_mu_bar_bootstrap90']}; operating at {bmu:.3f}")
    X = np.array(ins_feat, dtype=np.float32)
    ok = np.array([not r["flags"] & 0x3 and math.isfinite(r["dH"]) for r in ins_recs])
    y = -beta * np.array([r["dH"] for r in ins_recs])[ok]
    X = X[ok]
    y = y - y.mean()
    sd = y.std()
    y = np.clip(y, -8.0 * sd, 8.0 * sd).astype(np.float32)
    cap = float(y.max())
    t0 = time.perf_counter()
    oof = out_of_fold(h4d, X, y, args.train_epochs)
    net, steps, losses = train_network(h4d, X, y, args.train_epochs)
    train_s = time.perf_counter() - t0
    oof_corr = float(np.corrcoef(oof, y)[0, 1]) if np.std(oof) > 0 else None
    note(f"{label}: network: out-of-fold correlation {oof_corr}")
    one.set_beta_mu(bmu)
    scale = args.scale
    select = None
    if scale is None:
        arms = {"plain": (None, 0, 0.0, cap)}
        for sc in (0.25, 0.5, 1.0):
            arms[f"scale{sc}"] = (net, candidates, sc, cap)
        select = proposal_ab(one, torch, h4d, arms, bmu, n_select)
        best, best_v = 0.0, select["plain"]["log10_expected_exchanges_per_s"] + math.log10(1.25)
        for sc in (0.25, 0.5, 1.0):
            v = select[f"scale{sc}"]["log10_expected_exchanges_per_s"]
            if v > best_v:
                best, best_v = sc, v
        scale = best
    note(f"{label}: weight scale {scale} at k = {candidates}")
    ab = None
    if n_ab > 0:
        ab = proposal_ab(one, torch, h4d, {"plain": (None, 0, 0.0, cap), "learned": (net, candidates, scale, cap)},
                         bmu, n_ab)
    one.close()
    info = {"candidates": candidates, "weight_scale": scale, "logit_cap": cap,
            "inference": "BF16 MFMA (v_mfma_f32_16x16x16_bf16), FP32 accumulation",
            "target": "-beta dH of the pilot insertions, centred, clipped to 8 standard deviations",
            "out_of_fold_corr_logit_vs_target": oof_corr, "target_sd_kT": float(sd),
            "pilot_insertions": n_ins, "pilot_deletions": n_del, "pilot_s": pilot_s,
            "train_rows": int(len(X)), "train_steps": steps, "train_s": train_s,
            "train_loss_first": float(losses[:10].mean()), "train_loss_last": float(losses[-50:].mean()),
            "scale_selection": select, "fixed_state": ab}
    return net, scale, cap, over, info, cal, bmu


def bias_study(h4d, torch, w, beta_mu, n_each, x_b, alpha_b, v_ex):
    """The bimodal bias of the flyers' separation (Sec. II B 4, Eq. 14) and
    early rejection on top of it, against the uniform proposal, at a fixed
    state (proposal_ab)."""
    one = h4d.System.from_workload(w)
    try:
        return proposal_ab(one, torch, h4d, {"plain": (None, 0, 0.0, 0.0),
                                              "bias": (None, 0, 0.0, 0.0, (x_b, alpha_b, 0.0)),
                                              "bias_early": (None, 0, 0.0, 0.0, (x_b, alpha_b, v_ex))},
                           beta_mu, n_each)
    finally:
        one.close()


# ---------------------------------------------------------------------------
# The default workload: aqueous NaCl, learned vs plain
# ---------------------------------------------------------------------------
def timed_arms(args, h4d, torch, w, beta_mu, over, net, scale, cap, candidates, steps, warmup, timing_trials):
    """The plain and learned arms, each one chain from the same state on
    speculative replicas; returns their summaries and the learned arm's
    step-kernel timing."""
    arms, timing = {}, None
    for name in ("plain", "learned"):
        spec = h4d.Speculative.from_workload(w, args.replicas, beta_mu=beta_mu, **over)
        if name == "learned" and scale > 0.0:
            spec.set_proposal(net, candidates, cap, scale)
        if warmup:
            spec.trials(warmup)
        r0 = spec.rounds
        arr, wall = timed(torch, lambda: spec.trials(steps, as_array=True))
        arms[name] = arm_summary([arr[q] for q in range(steps)], wall, spec.rounds - r0)
        note(f"{name}: {steps} trials in {wall:.2f} s, {arms[name]['accepted']} accepted")
        if name == "learned" and timing_trials > 0:
            spec.set_timing(True)
            spec.trials(timing_trials)
            timing = spec.timing()
            spec.set_timing(False)
        spec.close()
    return arms, timing


def learned_vs_plain(arms, info):
    la, pa = arms["learned"], arms["plain"]
    fs = (info or {}).get("fixed_state") or {}
    curve = None
    if "plain" in fs and "learned" in fs:
        lp, ll = fs["plain"]["log10_p_insert_at_beta_mu_plus"], fs["learned"]["log10_p_insert_at_beta_mu_plus"]
        curve = {sh: (ll[sh] - lp[sh] if math.isfinite(ll[sh]) and math.isfinite(lp[sh]) else None) for sh in lp}
    return {
        "fixed_state_insertion_log10_gain_at_beta_mu_plus": curve,
        "accepted_exchanges_per_s_ratio": (la["accepted_exchanges_per_s"] / pa["accepted_exchanges_per_s"]
                                           if pa["accepted"] > 0 else None),
        "expected_exchanges_per_s_ratio": (la["expected_exchanges_per_s"] / pa["expected_exchanges_per_s"]
                                           if pa["expected_exchanges_per_s"] > 1e-300 else None),
        "atom_steps_per_s_ratio": la["atom_steps_per_s"] / pa["atom_steps_per_s"],
        "fixed_state_log10_gain": ((info or {}).get("fixed_state") or {}).get("log10_gain_learned"),
        "fixed_state_log10_gain_bootstrap90": ((info or {}).get("fixed_state") or {}).get(
            "log10_gain_learned_bootstrap90"),
    }


def gcmd_cycles(args, h4d, torch, w, beta_mu, over, cycles, n_eq):
    """The grand-canonical cycle of Fig. 1 on one box: an equilibrium phase
    of n_eq steps (generalized hybrid MC, partial momentum refresh c = 0.5)
    and one exchange trial that carries the state's momenta with the
    symmetric two-end reversal (Sec. II A)."""
    g = h4d.System.from_workload(w, beta_mu=beta_mu, momenta=1, md_refresh=0.5, **over)
    g.md_phase(n_eq)
    g.trial()
    md, tr = [], []
    t_md = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(cycles):
        t1 = time.perf_counter()
        md.append(g.md_phase(n_eq)[0])
        torch.cuda.synchronize()
        t_md += time.perf_counter() - t1
        tr.append(g.trial())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    steps = sum(r["n_atoms"] * (r["n_steps"] + 1) for r in md + tr)
    note(f"gcmd: {cycles} cycles of {n_eq} equilibrium steps and one trial in {wall:.2f} s")
    return {"cycle": f"equilibrium phase of {n_eq} steps (partial momentum refresh c = 0.5, Metropolis on dH) + "
                     "one trial with carried momenta and the two-end reversal",
            "cycles": cycles, "ms_per_cycle": 1e3 * wall / cycles, "atom_steps_per_s": steps / wall,
            "equilibrium_share_of_wall": t_md / wall,
            "equilibrium_acceptance": sum(r["accepted"] for r in md) / cycles,
            "equilibrium_mean_abs_beta_dH": sum(abs(r["dH"]) for r in md) / cycles / w.params["kT"],
            "trials_accepted": sum(r["accepted"] for r in tr)}


def bench_nacl(args, h4d, W, torch):
    w0 = W.config_water_nacl()
    w0.params.update(capacity=w0.n + 1024)
    if args.skin is not None:   # Verlet skin (A); trajectories depend on it only through the summation order
        w0.params.update(skin=args.skin)
    w = relaxed(h4d, w0, args.relax_phases, 100) if args.relax_phases > 0 else w0
    if args.pilot > 0:
        net, scale, cap, over, info, cal, beta_mu = learned_study(
            args, h4d, torch, w, "nacl", args.pilot, args.pilot_del, args.select_trials, args.ab_trials,
            args.candidates, beta_mu=args.beta_mu)
    else:   # no pilot, no network: both arms uniform (a profiling run of the timed configuration)
        if args.beta_mu is None:
            raise SystemExit("bench.py: --pilot 0 needs --beta-mu")
        net, scale, cap, info, cal, beta_mu = None, 0.0, 10.0, None, None, args.beta_mu
        over = {"lanes_per_atom": args.lanes} if args.lanes else {}
    arms, timing = timed_arms(args, h4d, torch, w, beta_mu, over, net, scale, cap, args.candidates, args.steps,
                              args.warmup, args.timing_trials)
    if net is not None:
        net.close()
    gcmd = gcmd_cycles(args, h4d, torch, w, beta_mu, over, args.gcmd_cycles, 1000) if args.gcmd_cycles else None
    la = arms["learned"]
    out = {
        "value": la["atom_steps_per_s"], "trials_per_s": la["trials_per_s"],
        "accepted_exchanges_per_s": la["accepted_exchanges_per_s"],
        "arms": arms,
        "learned_vs_plain": dict(learned_vs_plain(arms, info), note=(
            "at the BAR beta mu with 500-step flights of 0.5 ps, neither proposal's exchanges are accepted in a "
            "bench-length run; the fixed-state comparison gives their expected acceptance in log space")),
        "learned": info,
        "mu_calibration": cal,
        "gcmd": gcmd,
        "roofline": roofline(timing, counted_traffic("water", timing),
                             "k_step<1,L> (fused pair force + velocity Verlet), learned arm",
                             counted_valu_busy("water", timing)),
        "lanes_per_atom": timing["lanes"], "rebuild_every": timing["rebuild_every"],
        "nontemporal_lists": timing["nt_lists"],
        "execution": {"mode": "speculative", "replicas": args.replicas},
    }
    config = {
        "workload": "aqueous NaCl + learned proposal: 8,000 rigid SPC/E waters + 150 NaCl pairs in a 62 A box, "
                    "298 K, 500-step NEMD NaCl-pair insert/delete (dt 1 fs, w_max 3 A, kappa_sr 1/A, DSF alpha "
                    "0.25/A cut 10 A), FP32 pair arithmetic / FP64 state, energies and work; learned arm: "
                    f"multiple-try over {args.candidates} candidate sites scored by a 64-3x128-1 network (BF16), "
                    f"plain arm: uniform; each arm one chain on {args.replicas} speculative replicas",
        "n_atoms": w.n, "n_waters": 8000, "n_pairs": 150, "box_A": 62.0, "n_steps_per_trial": 500,
        "dt_fs": 1.0, "w_max_A": 3.0, "candidates": args.candidates,
        "start": f"lattice start relaxed by {args.relax_phases} equilibrium phases of 100 steps",
        "beta_mu": beta_mu, "beta_mu_source": "given" if args.beta_mu is not None else
        "Bennett's acceptance ratio over the pilot insertions and deletions",
        "skin": w.params["skin"], "parallelism": f"one chain, {args.replicas} speculative replicas, one GPU",
    }
    base = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_steps or 60, "the aqueous NaCl state",
                                                          beta_mu)
    return out, config, base


# ---------------------------------------------------------------------------
# The 32,000-ion LJ chain and the 256-box batch
# ---------------------------------------------------------------------------
def leg_lj32k(args, h4d, W, torch, steps, warmup, timing_trials):
    """The 32,000-ion LJ chain (relaxed lattice start) at its BAR beta mu:
    plain and learned arms on speculative replicas, and the learned study
    behind them."""
    w0 = W.config_lj_32k()
    w0.params.update(capacity=w0.n + 1024)
    w = relaxed(h4d, w0, args.lj_relax_phases, 200) if args.lj_relax_phases > 0 else w0
    if args.lj_pilot > 0:
        net, scale, cap, over, info, cal, bmu = learned_study(
            args, h4d, torch, w, "lj32k", args.lj_pilot, args.lj_pilot // 2, args.select_trials, args.lj_ab_trials,
            args.candidates, beta_mu=args.lj_beta_mu)
    else:   # no pilot, no network: both arms uniform (a profiling run of the timed configuration)
        if args.lj_beta_mu is None:
            raise SystemExit("bench.py: --lj-pilot 0 needs --lj-beta-mu")
        net, scale, cap, info, cal, bmu = None, 0.0, 10.0, None, None, args.lj_beta_mu
        over = {"lanes_per_atom": args.lanes} if args.lanes else {}
    arms, tm = timed_arms(args, h4d, torch, w, bmu, over, net, scale, cap, args.candidates, steps, warmup,
                          timing_trials)
    if net is not None:
        net.close()
    bias = None
    if args.lj_bias_trials > 0:
        # flyers near contact (x_b = 1 sigma, alpha_b = 2 / sigma^2); V_ex edge 1.2 sigma
        bias = bias_study(h4d, torch, w, bmu, args.lj_bias_trials, 1.0, 2.0, 1.2)
        bias["settings"] = {"x_b": 1.0, "alpha_b": 2.0, "v_ex_edge": 1.2}
        note(f"lj32k: bias: log10 gain {bias['log10_gain_bias']} {bias['log10_gain_bias_bootstrap90']}, "
             f"with early rejection {bias['log10_gain_bias_early']}")
    out = dict(arms["plain"])
    out["value"] = out.pop("atom_steps_per_s")
    out["learned_arm"] = arms["learned"]
    out["learned_vs_plain"] = learned_vs_plain(arms, info)
    out["learned"] = info
    out["mu_calibration"] = cal
    out["bimodal_bias"] = bias
    out["roofline"] = roofline(tm, counted_traffic("lj32k", tm),
                               "k_step<1,L> (fused pair force + velocity Verlet)")
    out["lanes_per_atom"], out["rebuild_every"] = tm["lanes"], tm["rebuild_every"]
    out["nontemporal_lists"] = tm["nt_lists"]
    out["config"] = {"workload": "lj32k: 32,000 LJ ions, density 0.3, 200-step NEMD pair insert/delete, FP32 pair "
                                 "arithmetic / FP64 state; value: the uniform proposal, one chain on speculative "
                                 "replicas; learned_arm: the same chain with the learned multiple-try proposal",
                     "replicas": args.replicas, "beta_mu": bmu, "start": f"lattice start relaxed by "
                     f"{args.lj_relax_phases} equilibrium phases of 200 steps", "candidates": args.candidates}
    note(f"lj32k: {steps} trials per arm, {out['value']:.3g} atom-steps/s, frac {out['roofline']['frac']:.3f}")
    return out, w


def leg_lj500(args, h4d, W, torch, trials=100):
    """The 500-ion FP64 box (the smallest LJ configuration): latency-bound,
    so microseconds per step rather than a roofline.  One chain, one trial
    after another, from a relaxed start; every kernel of a trial is one
    graph replay."""
    w = relaxed(h4d, W.config_lj_500(), 5, 200)
    g = h4d.System.from_workload(w)
    g.trials(5)
    arr, wall = timed(torch, lambda: g.trials(trials, as_array=True))
    recs = [arr[q] for q in range(trials)]
    g.close()
    out = arm_summary(recs, wall)
    launches = sum(r.n_steps + 1 for r in recs)
    out["us_per_step"] = 1e6 * wall / max(1, launches)
    out["config"] = {"workload": "lj500: 500 LJ ions (250 +1 / 250 -1), density 0.3, 100-step NEMD pair insert/delete, "
                                 "dt 0.005, w_max 2.5 sigma, FP64; one chain, one trial after another",
                     "beta_mu": w.params["beta_mu"], "start": "random start relaxed by 5 equilibrium phases of 200 steps"}
    note(f"lj500: {trials} trials, {out['us_per_step']:.1f} us per step, {out['accepted']} accepted")
    return out


# Trials per box of the 256-box workload after the autotuner, as far as it has
# run without fault on the GPU (33 rounds of one handle in all, the autotuner's
# 26 included).
BATCHED_MAX_TRIALS = 7


def leg_batched(args, h4d, W, torch, steps, warmup, timing_trials, learned_k=0):
    ws = W.config_batched()
    for w in ws:
        w.params.update(beta_mu=args.batch_beta_mu)
        if args.fixed_nf:     # every trial the same N_f: rounds with no box idle, for comparison
            w.params.update(n_steps_min=args.fixed_nf, n_steps_max=args.fixed_nf)
        if args.rebuild_every:
            w.params.update(rebuild_every=args.rebuild_every)
        if args.lanes:
            w.params.update(lanes_per_atom=args.lanes)
    bat = h4d.Batch.from_workloads(ws)
    tuned = bat.autotune(1) if args.autotune else None
    if warmup:
        bat.run(warmup)
    arr, wall = timed(torch, lambda: bat.run(steps, as_array=True))
    recs = [arr[q] for q in range(len(ws) * steps)]
    out = arm_summary(recs, wall)
    # lockstep rounds: round q runs trial q of every box for as many steps as
    # its longest trajectory; the share of those atom-step slots that integrate
    work = slots = 0
    for q in range(steps):
        rr = [arr[b * steps + q] for b in range(len(ws))]
        work += sum(r.n_steps * r.n_atoms for r in rr)
        slots += max(r.n_steps for r in rr) * sum(r.n_atoms for r in rr)
    out["lockstep_slot_utilisation"] = work / max(1, slots)
    bat.set_timing(True)
    bat.run(timing_trials)
    tm = bat.timing()
    bat.close()
    out["value"] = out.pop("atom_steps_per_s")
    out["roofline"] = roofline(tm, counted_traffic("batched", tm),
                               "k_step<1,L> (fused pair force + velocity Verlet)")
    out["lanes_per_atom"], out["rebuild_every"] = tm["lanes"], tm["rebuild_every"]
    out["nontemporal_lists"] = tm["nt_lists"]
    # over the handle's whole life, the autotuner's trials included
    out["handle_nonfinite_trials"], out["handle_retried_trials"] = tm["nonfinite"], tm["retries_total"]
    out["list_capacity"] = {"entries_per_atom": tm["nbr_cap"], "atoms_per_cell": tm["cell_cap"]}
    out["autotune"] = tuned
    out["config"] = {"workload": "batched256: 256 LJ-electrolyte boxes, N even in [1000, 16000] (2,220,126 ions), "
                                 "density U[0.1, 0.4], N_f ~ U{100..400} per trial, FP32 pair arithmetic / FP64 "
                                 "state, uniform proposal; every box runs its trial in one round of launches" +
                                 (f" (N_f fixed at {args.fixed_nf} for comparison)" if args.fixed_nf else ""),
                     "n_boxes": len(ws), "n_atoms": sum(w.n for w in ws), "trials_per_box": steps,
                     "beta_mu": args.batch_beta_mu}
    note(f"batched256: {steps} trials per box, {out['value']:.3g} atom-steps/s, frac {out['roofline']['frac']:.3f}")
    return out, ws


def batched_learned_vs_plain(args, h4d, W, torch, trials, k=256, scales=(0.5, 1.0), pilot_boxes=16,
                             pilot_per_box=64):
    """The 256-box batch with the learned proposal against the uniform one:
    a network trained on forced uniform insertions in 16 of the boxes (spread
    over their density range, one box at a time), then one fresh batch per
    arm from the same start state running `trials` trials per box at the
    workload's beta mu, where insertions are often accepted: accepted
    exchanges per second and the insertion and deletion acceptances with
    their Wilson intervals."""
    import numpy as np
    ws = W.config_batched()
    for w in ws:
        w.params.update(beta_mu=args.batch_beta_mu, lanes_per_atom=4)
    beta = 1.0 / ws[0].params["kT"]
    dens = np.array([w.n / np.prod(w.params["box"]) for w in ws])
    pick = np.argsort(dens)[np.linspace(0, len(ws) - 1, pilot_boxes).astype(int)]
    X, y = [], []
    t0 = time.perf_counter()
    for b in pick:
        one = h4d.System.from_workload(ws[int(b)])
        recs, feats, _ = pilot(one, h4d, pilot_per_box, 0)["ins"]
        one.close()
        for r, f in zip(recs, feats):
            if not r["flags"] & 0x3 and math.isfinite(r["dH"]):
                X.append(f)
                y.append(-beta * r["dH"])
    pilot_s = time.perf_counter() - t0
    X = np.array(X, dtype=np.float32)
    y = np.array(y)
    y = y - y.mean()
    sd = y.std()
    y = np.clip(y, -8.0 * sd, 8.0 * sd).astype(np.float32)
    cap = float(y.max())
    oof = out_of_fold(h4d, X, y, args.train_epochs)
    net, _, _ = train_network(h4d, X, y, args.train_epochs)
    oof_corr = float(np.corrcoef(oof, y)[0, 1]) if np.std(oof) > 0 else None
    arms = {}
    for name, scale in [("plain", 0.0)] + [(f"learned_scale{sc}", sc) for sc in scales]:
        bat = h4d.Batch.from_workloads(ws)
        if scale > 0.0:
            bat.set_proposal(net, k, cap, scale)
        arr, wall = timed(torch, lambda: bat.run(trials, as_array=True))
        arms[name] = arm_summary([arr[q] for q in range(len(ws) * trials)], wall)
        arms[name]["value"] = arms[name].pop("atom_steps_per_s")
        bat.close()
        note(f"batched256 {name}: {arms[name]['accepted']} of {arms[name]['trials']} accepted, "
             f"{arms[name]['accepted_exchanges_per_s']:.1f} exchanges/s")
    net.close()
    pa = arms["plain"]
    return {
        "pilot": {"boxes": [int(b) for b in pick], "insertions": int(len(y)), "seconds": pilot_s,
                  "out_of_fold_correlation": oof_corr},
        "candidates": k, "trials_per_box": trials, "beta_mu": args.batch_beta_mu,
        "arms": arms,
        "accepted_exchanges_per_s_ratio": {name: (a["accepted_exchanges_per_s"] / pa["accepted_exchanges_per_s"]
                                                  if pa["accepted"] > 0 else None)
                                           for name, a in arms.items() if name != "plain"},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("nacl", "lj32k", "batched"), default="nacl")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed exchange trials per arm (nacl, default 24), of the chain (lj32k, default 400) or "
                         "per box (batched, default 4; warmup + steps + timing trials at most 7)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed trials first (default 5 / 20 / 2)")
    ap.add_argument("--beta-mu", type=float, default=None,
                    help="nacl: beta mu (default: Bennett's acceptance ratio over the pilot moves)")
    ap.add_argument("--lj-beta-mu", type=float, default=None,
                    help="lj32k: beta mu (default: Bennett's acceptance ratio over its pilot moves)")
    ap.add_argument("--lj-pilot", type=int, default=1000, help="lj32k: pilot insertions (half as many deletions)")
    ap.add_argument("--lj-relax-phases", type=int, default=10,
                    help="lj32k: equilibrium phases of 200 steps that relax the lattice start")
    ap.add_argument("--lj-bias-trials", type=int, default=150,
                    help="lj32k: forced insertions and deletions per arm of the bimodal-bias comparison (0: none)")
    ap.add_argument("--lj-ab-trials", type=int, default=300,
                    help="lj32k: forced insertions and deletions per proposal in the fixed-state comparison")
    ap.add_argument("--relax-phases", type=int, default=40,
                    help="nacl: equilibrium phases of 100 steps that relax the lattice start")
    ap.add_argument("--gcmd-cycles", type=int, default=3,
                    help="nacl: grand-canonical cycles (1000-step equilibrium phase + one trial) timed after the rest")
    ap.add_argument("--select-trials", type=int, default=60,
                    help="forced insertions and deletions per weight scale when choosing it")
    ap.add_argument("--batch-beta-mu", type=float, default=-4.0, help="batched: beta mu")
    ap.add_argument("--batch-learned-trials", type=int, default=4,
                    help="batched: trials per box of each arm of the learned-vs-plain comparison (0: none)")
    ap.add_argument("--fixed-nf", type=int, default=0,
                    help="batched: every trial N_f steps (0: N_f ~ U{100..400} per trial, the workload's own)")
    ap.add_argument("--pilot", type=int, default=2000,
                    help="nacl: pilot insertions (0: no learned study, both arms uniform; needs --beta-mu)")
    ap.add_argument("--pilot-del", type=int, default=1000, help="nacl: pilot deletions")
    ap.add_argument("--train-epochs", type=int, default=30, help="nacl: passes over the pilot data")
    ap.add_argument("--candidates", type=int, default=CANDIDATES, help="nacl: candidate sites per learned move")
    ap.add_argument("--scale", type=float, default=None, help="nacl: weight scale (default: chosen from the pilot)")
    ap.add_argument("--replicas", type=int, default=8, help="speculative replicas of a single chain")
    ap.add_argument("--ab-trials", type=int, default=200,
                    help="nacl: forced insertions and deletions per proposal on the start state (0: none)")
    ap.add_argument("--timing-trials", type=int, default=None,
                    help="trials after the timed region with HIP events on the step kernel (default 4 / 20 / 1)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle sample length (N_f of its one trial; default 60 for nacl, the full flight for lj32k)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="nacl: leave out the lj32k and batched keys")
    ap.add_argument("--rebuild-every", type=int, default=0, help="list rebuild interval (0: library default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: library default)")
    ap.add_argument("--skin", type=float, default=None, help="nacl: Verlet skin in A (default: the workload's)")
    ap.add_argument("--autotune-trials", type=int, default=4,
                    help="trials the autotuner times per choice of the single-chain legs")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library's lanes per atom and automatic rebuild interval")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the stream-copy probe on MIB mebibytes and print its bandwidth")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "boxes are independent Markov chains and would shard across GPUs without communication, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    wl = args.workload
    if args.steps is None:
        # nacl: three whole rounds of the default 8 speculative replicas (a
        # partial last round would run replicas past the timed trials)
        args.steps = {"nacl": 24, "lj32k": 400, "batched": 4}[wl]
    if args.warmup is None:
        args.warmup = {"nacl": 5, "lj32k": 20, "batched": 2}[wl]
    if args.timing_trials is None:
        args.timing_trials = {"nacl": 4, "lj32k": 20, "batched": 1}[wl]
    if args.batch_learned_trials > BATCHED_MAX_TRIALS or (
            wl == "batched" and args.warmup + args.steps + args.timing_trials > BATCHED_MAX_TRIALS):
        print(f"bench.py: the 256-box workload runs at most {BATCHED_MAX_TRIALS} trials per box after the "
              "autotuner (warmup + steps + timing trials): longer runs of it have faulted the GPU and the "
              "cause is not established", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_11447_amd import h4d
    from paper_2307_11447_amd import workloads as W

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        ms = h4d.stream_copy(nbytes, 20)
        print(json.dumps({"probe": "stream_copy", "bytes": nbytes, "ms": ms,
                          "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return

    extras = {}
    if wl == "nacl":
        out, config, base = bench_nacl(args, h4d, W, torch)
        if not args.no_extras:
            extras["lj32k"], w32 = leg_lj32k(args, h4d, W, torch, 200, 10, 5)
            if not args.no_cpu_baseline:
                extras["lj32k"]["cpu_baseline"] = cpu_baseline(w32, 200, "the 32,000-ion state",
                                                               extras["lj32k"]["config"]["beta_mu"])
            extras["batched256"], _ = leg_batched(args, h4d, W, torch, 2, 1, 1)
            if args.batch_learned_trials > 0:
                extras["batched256"]["learned_vs_plain"] = batched_learned_vs_plain(args, h4d, W, torch,
                                                                                    args.batch_learned_trials)
            extras["lj500"] = leg_lj500(args, h4d, W, torch)
    elif wl == "lj32k":
        out, w32 = leg_lj32k(args, h4d, W, torch, args.steps, args.warmup, args.timing_trials)
        config = out.pop("config")
        base = None if args.no_cpu_baseline else cpu_baseline(w32, args.cpu_steps or 200, "the 32,000-ion state",
                                                              config["beta_mu"])
    else:
        out, ws = leg_batched(args, h4d, W, torch, args.steps, args.warmup, args.timing_trials)
        if args.batch_learned_trials > 0:
            out["learned_vs_plain"] = batched_learned_vs_plain(args, h4d, W, torch, args.batch_learned_trials)
        config = out.pop("config")
        big = max(ws, key=lambda w: w.n)
        base = None if args.no_cpu_baseline else cpu_baseline(big, args.cpu_steps or 100,
                                                              f"the largest box ({big.n} ions)", args.batch_beta_mu)
    n_boxes = config.get("n_boxes", 1)
    line = {
        "metric": METRIC,
        "value": out.pop("value"),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / out["trials_per_s"] * n_boxes,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": config,
    }
    line.update(out)
    line.update(extras)
    if base is not None:
        line["cpu_baseline"] = base
    print(json.dumps(finite_json(line)), flush=True)


if __name__ == "__main__":
    main()
