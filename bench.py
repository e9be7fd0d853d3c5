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
Before the timed region: pilot insertions and deletions on the start state
(forced moves that are never accepted, so the state stays fixed) give the
operating beta mu by Bennett's acceptance ratio (Crooks' relation, the
supplement's CFT/BAR section) and the network's training data (features and
work of the method's own moves); the network trains on the GPU (FP32
forward, backward, Adam).

One "step" of this benchmark is one exchange trial of the chain.  value =
NEMD atom-steps/s of the learned arm (the whole hot path, candidate scoring
included); the plain arm, accepted exchanges/s of both arms with Wilson
intervals, and a fixed-state comparison of their insertion and deletion
acceptance stand beside it.  Extra keys time the 32,000-ion LJ chain and
the 256-box batch (--no-extras leaves them out).

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
TRAFFIC_FILES = {
    "water": os.path.join(ROOT, "profiles", "k_step_water_traffic.txt"),
    "lj32k": os.path.join(ROOT, "profiles", "k_step_lj32k_traffic.txt"),
    "batched": os.path.join(ROOT, "profiles", "k_step_batched256_traffic.txt"),
}
CANDIDATES = 4096


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


def counted_traffic(path):
    """HBM bytes per step launch from a committed rocprofv3 counter summary,
    or None if it is missing or was taken on different kernel sources."""
    from paper_2307_11447_amd import rocprof_summary
    if not path or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("kernel_source_sha256") != rocprof_summary.kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(timing, traffic_bytes, kernel):
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


def ln_ratio_at(rec, beta_mu_rec, beta_mu):
    """ln R of a record moved from the beta mu it ran at to another one
    (an insertion's ln R rises with beta mu, a deletion's falls)."""
    lr = rec["ln_ratio"]
    if rec["flags"] & 0x3 or not math.isfinite(lr):
        return -math.inf
    return lr + (beta_mu - beta_mu_rec) * (1.0 if rec["move"] > 0 else -1.0)


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


def choose_scale(s_ins, lr_ins, s_del, lr_del, cap=10.0, scales=(0.25, 0.5, 0.75, 1.0), margin=1.25):
    """Weight scale of the multiple-try proposal at many candidates, from
    uniform pilot moves: with k large, the chosen site is drawn from
    q(y) ~ exp(lw(y)) over uniform sites and ln(W/k) tends to ln Z,
    Z = E_uniform[exp(lw)], so the mean insertion acceptance is
    sum_i e^lw_i min(1, e^(lnR_i + lnZ - lw_i)) / sum_i e^lw_i (importance
    weights over the pilot insertions) and the mean deletion acceptance
    mean_j min(1, e^(lnR_j + lw_j - lnZ)); lw = scale min(s, cap), s the
    network's logits (out-of-fold for the insertions).  The uniform proposal
    (scale 0) is kept unless the best scale beats it by the margin."""
    import numpy as np
    s_ins = np.minimum(np.asarray(s_ins, np.float64), cap)
    s_del = np.minimum(np.asarray(s_del, np.float64), cap)
    lr_ins = np.asarray(lr_ins, np.float64)
    lr_del = np.asarray(lr_del, np.float64)

    def est(scale):
        lw_i, lw_d = scale * s_ins, scale * s_del
        m = lw_i.max()
        wi = np.exp(lw_i - m)
        lnZ = m + math.log(wi.mean())
        p_ins = float((wi * np.exp(np.minimum(0.0, lr_ins + lnZ - lw_i))).sum() / wi.sum())
        p_del = float(np.mean(np.exp(np.minimum(0.0, lr_del + lw_d - lnZ))))
        return p_ins, p_del

    table = {"uniform": est(0.0)}
    best, best_v = 0.0, 0.5 * sum(table["uniform"]) * margin
    for sc in scales:
        table[f"scale{sc}"] = est(sc)
        v = 0.5 * sum(table[f"scale{sc}"])
        if v > best_v:
            best, best_v = sc, v
    return best, {k: {"p_ins": v[0], "p_del": v[1]} for k, v in table.items()}


def proposal_ab(sys_, torch, h4d, arms, beta_mu, n_each, block=50):
    """Insertion and deletion acceptance of several proposals on one fixed
    state: forced moves at beta mu = -1000 (insertions) and +1000
    (deletions), which are never accepted, so the state does not change;
    each record's ln R is moved to the operating beta mu and the mean of
    min(1, R) taken.  The arms alternate in blocks so that they share the
    same state and device conditions.  arms: name -> (net, k, scale)."""
    out = {name: {"ins": [], "del": [], "s": 0.0, "n": 0} for name in arms}
    done = 0
    while done < n_each:
        nb = min(block, n_each - done)
        for name, (net, k, scale) in arms.items():
            if k > 0:
                sys_.set_proposal(net, k, 10.0, scale)
            else:
                sys_.set_proposal(None, 0)
            for move, bm, key in ((h4d.MOVE_INSERT, -1.0e3, "ins"), (h4d.MOVE_DELETE, 1.0e3, "del")):
                sys_.set_beta_mu(bm)
                arr, dt = timed(torch, lambda: sys_.trials(nb, move, as_array=True))
                out[name]["s"] += dt
                out[name]["n"] += nb
                shift = (beta_mu - bm) * (1.0 if move > 0 else -1.0)
                for q in range(nb):
                    r = arr[q]
                    ok = not (r.flags & 0x3) and math.isfinite(r.ln_ratio)
                    out[name][key].append(math.exp(min(0.0, r.ln_ratio + shift)) if ok else 0.0)
        done += nb
    sys_.set_proposal(None, 0)
    sys_.set_beta_mu(beta_mu)
    res = {}
    for name, o in out.items():
        p_ins = sum(o["ins"]) / max(1, len(o["ins"]))
        p_del = sum(o["del"]) / max(1, len(o["del"]))
        rate = o["n"] / max(1e-300, o["s"])
        res[name] = {"p_insert": p_ins, "p_delete": p_del, "trials_per_s": rate,
                     "expected_exchanges_per_s": 0.5 * (p_ins + p_del) * rate,
                     "insertions": len(o["ins"]), "deletions": len(o["del"])}
    names = list(arms)
    for other in names[1:]:
        g, ci = ab_gain(out[names[0]], out[other])
        res[f"gain_{other}"], res[f"gain_{other}_bootstrap90"] = g, ci
    return res


def ab_gain(u, l, reps=2000, seed=11):
    """Ratio of expected exchanges per second (another proposal over the
    first) and its 90 % bootstrap interval (moves resampled within each arm
    and kind); None when the first arm's expected acceptance is below 1e-12
    (the ratio is then meaningless)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    rate_u, rate_l = u["n"] / u["s"], l["n"] / l["s"]

    def ex(o, rate, pick):
        return 0.5 * (np.mean(pick(o["ins"])) + np.mean(pick(o["del"]))) * rate

    ident = np.asarray
    if ex(u, rate_u, ident) < 1e-12:
        return None, None
    g = ex(l, rate_l, ident) / ex(u, rate_u, ident)
    boot = []
    for _ in range(reps):
        def res(x):
            x = np.asarray(x)
            return x[rng.integers(0, len(x), len(x))]
        den = ex(u, rate_u, res)
        boot.append(ex(l, rate_l, res) / den if den > 0 else float("inf"))
    lo, hi = np.percentile(boot, [5, 95])
    return float(g), [float(lo), float(hi)]


# ---------------------------------------------------------------------------
# The default workload: aqueous NaCl, learned vs plain
# ---------------------------------------------------------------------------
def bench_nacl(args, h4d, W, torch):
    import numpy as np
    from paper_2307_11447_amd import analysis
    w = W.config_water_nacl()
    w.params.update(capacity=w.n + 1024)
    beta = 1.0 / w.params["kT"]
    V = float(np.prod(w.params["box"]))
    one = h4d.System.from_workload(w)
    tuned = one.autotune(2) if args.autotune else None
    if tuned:
        note(f"autotune: {tuned[0]} lanes per atom, rebuild every {tuned[1]} steps")
    over = {}
    if tuned:
        over.update(lanes_per_atom=tuned[0], rebuild_every=tuned[1])
    # pilot on the start state (the autotuner's trials left it unchanged
    # unless one was accepted: take the state as it is now)
    st = one.state()
    t0 = time.perf_counter()
    pil = pilot(one, h4d, args.pilot, args.pilot_del)
    pilot_s = time.perf_counter() - t0
    note(f"pilot: {args.pilot} insertions and {args.pilot_del} deletions in {pilot_s:.1f} s")
    ins_recs, ins_feat, bm_ins = pil["ins"]
    del_recs, del_feat, bm_del = pil["del"]
    dM_ins = [r["dM"] for r in ins_recs if not r["flags"] & 0x3]
    dM_del = [r["dM"] for r in del_recs if not r["flags"] & 0x3]
    cal = analysis.work_summary(dM_ins, dM_del, beta, 0.0)
    beta_mu = args.beta_mu if args.beta_mu is not None else cal["beta_mu_bar"]
    cal = analysis.work_summary(dM_ins, dM_del, beta, beta_mu)
    cal["note"] = ("uniform forced insertions and deletions on the start state (none accepted): beta mu from "
                   "Bennett's acceptance ratio, P_acc predicted by Eq. (21) at the operating beta mu")
    note(f"BAR: beta mu = {cal['beta_mu_bar']:.3f} {cal['beta_mu_bar_bootstrap90']}; operating at {beta_mu:.3f}")
    # the network: target the clipped log insertion ratio at the operating
    # point, c - beta dH with c = beta mu + I
    c = beta_mu + 2.0 * math.log(V / (st["nsalt"] + 1))
    X = np.array(ins_feat, dtype=np.float32)
    bdH = beta * np.array([r["dH"] for r in ins_recs])
    ok = np.isfinite(bdH) & np.array([not r["flags"] & 0x3 for r in ins_recs])
    X, bdH = X[ok], bdH[ok]
    y = np.clip(c - bdH, -100.0, 10.0).astype(np.float32)
    t0 = time.perf_counter()
    oof = out_of_fold(h4d, X, y, args.train_epochs)
    net, steps, losses = train_network(h4d, X, y, args.train_epochs)
    s_del = net.forward(np.array(del_feat, dtype=np.float32))
    train_s = time.perf_counter() - t0
    lr_ins = [ln_ratio_at(r, bm_ins, beta_mu) for r, k in zip(ins_recs, ok) if k]
    lr_del = [ln_ratio_at(r, bm_del, beta_mu) for r in del_recs]
    scale, estimates = choose_scale(oof, lr_ins, s_del, lr_del)
    if args.scale is not None:
        scale = args.scale
    oof_corr = float(np.corrcoef(oof, y)[0, 1]) if np.std(oof) > 0 else None
    note(f"network: out-of-fold correlation {oof_corr}, weight scale {scale} at k = {args.candidates}")
    # the timed arms: the same chain from the same state on speculative replicas
    arms = {}
    learned_timing = None
    for name in ("plain", "learned"):
        spec = h4d.Speculative.from_workload(w, args.replicas, beta_mu=beta_mu, **over)
        if name == "learned":
            spec.set_proposal(net, args.candidates, 10.0, scale)
        if args.warmup:
            spec.trials(args.warmup)
        r0 = spec.rounds
        arr, wall = timed(torch, lambda: spec.trials(args.steps, as_array=True))
        recs = [arr[q] for q in range(args.steps)]
        arms[name] = arm_summary(recs, wall, spec.rounds - r0)
        note(f"{name}: {args.steps} trials in {wall:.2f} s, {arms[name]['accepted']} accepted")
        if name == "learned":
            spec.set_timing(True)
            spec.trials(args.timing_trials)
            learned_timing = spec.timing()
            spec.set_timing(False)
        spec.close()
    # both proposals on the start state, forced moves alternating in blocks
    ab = None
    if args.ab_trials > 0:
        one.set_beta_mu(beta_mu)
        ab = proposal_ab(one, torch, h4d, {"plain": (None, 0, 0.0), "learned": (net, args.candidates, scale)},
                         beta_mu, args.ab_trials)
        note(f"fixed-state comparison: {args.ab_trials} insertions and deletions per proposal")
    one.close()
    net.close()
    la, pa = arms["learned"], arms["plain"]
    out = {
        "value": la["atom_steps_per_s"], "trials_per_s": la["trials_per_s"],
        "accepted_exchanges_per_s": la["accepted_exchanges_per_s"],
        "arms": arms,
        "learned_vs_plain": {
            "accepted_exchanges_per_s_ratio": (la["accepted_exchanges_per_s"] / pa["accepted_exchanges_per_s"]
                                               if pa["accepted"] > 0 else None),
            "expected_exchanges_per_s_ratio": (la["expected_exchanges_per_s"] / pa["expected_exchanges_per_s"]
                                               if pa["expected_exchanges_per_s"] > 1e-12 else None),
            "atom_steps_per_s_ratio": la["atom_steps_per_s"] / pa["atom_steps_per_s"],
            "fixed_state": ab,
            "note": "accepted counts are rare at the BAR beta mu with 500-step flights; the expected acceptance "
                    "(mean of min(1, R) over the trials) and the fixed-state comparison carry the comparison",
        },
        "learned": {"candidates": args.candidates, "weight_scale": scale, "logit_cap": 10.0,
                    "inference": "BF16 MFMA (v_mfma_f32_16x16x16_bf16), FP32 accumulation",
                    "scale_choice_estimates": estimates, "out_of_fold_corr_logit_vs_target": oof_corr,
                    "pilot_insertions": args.pilot, "pilot_deletions": args.pilot_del, "pilot_s": pilot_s,
                    "train_rows": int(len(X)), "train_steps": steps, "train_s": train_s,
                    "train_loss_first": float(losses[:10].mean()), "train_loss_last": float(losses[-50:].mean()),
                    "target": "clip(beta mu + I - beta dH, -100, 10) of the pilot insertions"},
        "mu_calibration": cal,
        "roofline": roofline(learned_timing, counted_traffic(TRAFFIC_FILES["water"]),
                             "k_step<1,L> (fused pair force + velocity Verlet), learned arm"),
        "lanes_per_atom": learned_timing["lanes"], "rebuild_every": learned_timing["rebuild_every"],
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
    w = W.config_lj_32k()
    w.params.update(capacity=w.n + 1024, beta_mu=args.lj_beta_mu)
    spec = h4d.Speculative.from_workload(w, args.replicas)
    tuned = spec.autotune(2) if args.autotune else None
    if warmup:
        spec.trials(warmup)
    r0 = spec.rounds
    arr, wall = timed(torch, lambda: spec.trials(steps, as_array=True))
    out = arm_summary([arr[q] for q in range(steps)], wall, spec.rounds - r0)
    spec.set_timing(True)
    spec.trials(timing_trials)
    tm = spec.timing()
    spec.close()
    out["value"] = out.pop("atom_steps_per_s")
    out["roofline"] = roofline(tm, counted_traffic(TRAFFIC_FILES["lj32k"]),
                               "k_step<1,L> (fused pair force + velocity Verlet)")
    out["lanes_per_atom"], out["rebuild_every"] = tm["lanes"], tm["rebuild_every"]
    out["autotune"] = tuned
    out["config"] = {"workload": "lj32k: 32,000 LJ ions, density 0.3, 200-step NEMD pair insert/delete, FP32 pair "
                                 "arithmetic / FP64 state, uniform proposal, one chain on speculative replicas",
                     "replicas": args.replicas, "beta_mu": args.lj_beta_mu}
    note(f"lj32k: {steps} trials, {out['value']:.3g} atom-steps/s, frac {out['roofline']['frac']:.3f}")
    return out, w


def leg_batched(args, h4d, W, torch, steps, warmup, timing_trials, learned_k=0):
    ws = W.config_batched()
    for w in ws:
        w.params.update(beta_mu=args.batch_beta_mu)
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
    bat.set_timing(True)
    bat.run(timing_trials)
    tm = bat.timing()
    bat.close()
    out["value"] = out.pop("atom_steps_per_s")
    out["roofline"] = roofline(tm, counted_traffic(TRAFFIC_FILES["batched"]),
                               "k_step<1,L> (fused pair force + velocity Verlet)")
    out["lanes_per_atom"], out["rebuild_every"] = tm["lanes"], tm["rebuild_every"]
    out["autotune"] = tuned
    out["config"] = {"workload": "batched256: 256 LJ-electrolyte boxes, N even in [1000, 16000] (2,220,126 ions), "
                                 "density U[0.1, 0.4], N_f ~ U{100..400} per trial, FP32 pair arithmetic / FP64 "
                                 "state, uniform proposal; every box runs its trial in one round of launches",
                     "n_boxes": len(ws), "n_atoms": sum(w.n for w in ws), "trials_per_box": steps,
                     "beta_mu": args.batch_beta_mu}
    note(f"batched256: {steps} trials per box, {out['value']:.3g} atom-steps/s, frac {out['roofline']['frac']:.3f}")
    return out, ws


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("nacl", "lj32k", "batched"), default="nacl")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed exchange trials per arm (nacl, default 20), of the chain (lj32k, default 400) or "
                         "per box (batched, default 10)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed trials first (default 5 / 20 / 2)")
    ap.add_argument("--beta-mu", type=float, default=None,
                    help="nacl: beta mu (default: Bennett's acceptance ratio over the pilot moves)")
    ap.add_argument("--lj-beta-mu", type=float, default=-8.8,
                    help="lj32k: beta mu (default -8.8, the BAR estimate of the 32,000-ion state)")
    ap.add_argument("--batch-beta-mu", type=float, default=-4.0, help="batched: beta mu")
    ap.add_argument("--pilot", type=int, default=500, help="nacl: pilot insertions")
    ap.add_argument("--pilot-del", type=int, default=250, help="nacl: pilot deletions")
    ap.add_argument("--train-epochs", type=int, default=30, help="nacl: passes over the pilot data")
    ap.add_argument("--candidates", type=int, default=CANDIDATES, help="nacl: candidate sites per learned move")
    ap.add_argument("--scale", type=float, default=None, help="nacl: weight scale (default: chosen from the pilot)")
    ap.add_argument("--replicas", type=int, default=8, help="speculative replicas of a single chain")
    ap.add_argument("--ab-trials", type=int, default=150,
                    help="nacl: forced insertions and deletions per proposal on the start state (0: none)")
    ap.add_argument("--timing-trials", type=int, default=None,
                    help="trials after the timed region with HIP events on the step kernel (default 4 / 20 / 1)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle sample length (N_f of its one trial; default 60 for nacl, the full flight for lj32k)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="nacl: leave out the lj32k and batched keys")
    ap.add_argument("--rebuild-every", type=int, default=0, help="list rebuild interval (0: library default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: library default)")
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
        args.steps = {"nacl": 20, "lj32k": 400, "batched": 10}[wl]
    if args.warmup is None:
        args.warmup = {"nacl": 5, "lj32k": 20, "batched": 2}[wl]
    if args.timing_trials is None:
        args.timing_trials = {"nacl": 4, "lj32k": 20, "batched": 1}[wl]

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
            extras["lj32k"], w32 = leg_lj32k(args, h4d, W, torch, 100, 10, 5)
            if not args.no_cpu_baseline:
                extras["lj32k"]["cpu_baseline"] = cpu_baseline(w32, 200, "the 32,000-ion state",
                                                               args.lj_beta_mu)
            extras["batched256"], _ = leg_batched(args, h4d, W, torch, 2, 1, 1)
    elif wl == "lj32k":
        out, w32 = leg_lj32k(args, h4d, W, torch, args.steps, args.warmup, args.timing_trials)
        config = out.pop("config")
        base = None if args.no_cpu_baseline else cpu_baseline(w32, args.cpu_steps or 200, "the 32,000-ion state",
                                                              args.lj_beta_mu)
    else:
        out, ws = leg_batched(args, h4d, W, torch, args.steps, args.warmup, args.timing_trials)
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
