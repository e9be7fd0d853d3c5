#!/usr/bin/env python3
"""NEMD throughput of H4D salt-pair exchange trials on one MI355X.

Workload (N = 1): 32,000 Lennard-Jones ions (16,000 cations, 16,000
anions) at reduced density 0.3, T* = 1, Bjerrum length 3 sigma, LJ cut
2.5 sigma, damped shifted force Coulomb (alpha 0.3, cut 4 sigma); every
trial flies one cation-anion pair in or out along w in 200 velocity-Verlet
steps of dt = 0.005 (w_max = 2.5 sigma); FP32 pair arithmetic with FP64
positions, velocities, energies, work and Metropolis ratio; uniform
(plain) proposal.  One "step" of this benchmark is one exchange trial.

Prints one JSON line.  value = NEMD atom-steps/s (sum over trials of
atoms x N_f, divided by the wall time of the timed trials).

Both single-box workloads also measure the learned proposal: pilot
insertions give each uniform site's 64 features and dH, the network is
trained on them on the GPU, and the same number of timed trials run with
the multiple-try proposal it weights (reported under "learned", next to the
uniform run's accepted and expected exchanges per second).

--workload water: 8,000 rigid SPC/E waters + 150 NaCl pairs in a 62 A box,
NaCl-pair trials of 500 steps of 1 fs.

--workload batched: 256 independent boxes of 1,000-16,000 ions at
densities 0.1-0.4, N_f ~ U{100..400} per trial, all boxes running their
trials together; one "step" is one trial in every box.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted salt-pair exchanges/s + NEMD atom-steps/s (1 GPU), learned vs plain"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # published vector FP32 rate (packed FP32 counted)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_lj32k_traffic.txt")
TRAFFIC_FILE_BATCHED = os.path.join(ROOT, "profiles", "k_step_batched256_traffic.txt")


def counted_traffic(path):
    """HBM bytes per step launch from a committed rocprofv3 counter summary,
    or None if it is missing or was taken on different kernel sources."""
    from paper_2307_11447_amd import rocprof_summary
    if not os.path.exists(path):
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


def cpu_baseline(w, n_steps, label):
    """The FP64 oracle, single threaded, on a bounded sample: one trial of
    the given state with the trajectory cut to n_steps steps."""
    from oracle import build as ob
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        ob.build()
    params = dict(w.params, n_steps=n_steps, n_steps_min=0, n_steps_max=0)
    o = O.OracleSystem(params, w.x, w.type, w.mol, w.tag, w.nsalt, cap=w.n + 8)
    t0 = time.perf_counter()
    rec = o.trial(0)
    dt = time.perf_counter() - t0
    atoms = w.n
    return {"value": atoms * n_steps / dt, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 trial (move {rec['move']:+d}) of {label} with N_f cut to "
                      f"{n_steps} steps ({atoms * n_steps:.3g} atom-steps, {dt:.1f} s)"}


def step_bytes_per_atom(mean_nbr):
    """Algorithmic bytes of one fused step launch, per atom: 4 B per list
    entry, 4 B list length, 16 B own fixed-point record, 32 B own FP64
    position, 16 B fixed-point position at the list build, 64 B velocity in
    and out, 48 B new position (FP64 + fixed point); neighbour records are
    gathered through the caches and not counted."""
    return 4.0 * mean_nbr + 184.0


def step_flop_per_atom(mean_nbr):
    """Algorithmic floating-point operations of one fused step launch, per
    atom (an FMA counts 2, a reciprocal, square root or exponential 1).
    Per list entry, in FP32: the displacement and the squared 4D distance
    with the altitude term (9), the LJ force factor with 1/s^2 (7), the DSF
    Coulomb force factor with s, 1/s, the Gaussian and the erfc
    approximation (23), their sum (1) and the accumulation of the factor
    times the displacement (6): 46.  Per atom, in FP64: the two half kicks
    and the drift of velocity Verlet (18)."""
    return 46.0 * mean_nbr + 18.0


def summarize(recs, wall, timing, timing_recs, traffic_bytes, atom_launches=None):
    """Throughput, acceptance and the step kernel's roofline from trial
    records (recs: the timed trials; timing_recs: the trials run with HIP
    events around every step launch, or atom_launches: the atoms those
    launches integrated, summed over launches)."""
    n = len(recs)
    atom_steps = sum(r.n_atoms * r.n_steps for r in recs)
    acc = sum(r.accepted for r in recs)
    n_ins = sum(1 for r in recs if r.move > 0)
    n_ins_acc = sum(r.accepted for r in recs if r.move > 0)
    retried = sum(1 for r in recs if r.flags & 0x4)
    lo, hi = wilson(acc, n)
    mean_nbr = timing["mean_nbr"]
    bpa = step_bytes_per_atom(mean_nbr)
    # every step launch k = 0..N_f of a trial touches each of its atoms once
    if atom_launches is None:
        atom_launches = sum(r.n_atoms * (r.n_steps + 1) for r in timing_recs)
    step_s = timing["step_ms"] * 1e-3
    launches = max(1, timing["step_launches"])
    fpa = step_flop_per_atom(mean_nbr)
    achieved = fpa * atom_launches / step_s / 1e12
    achieved_bytes = bpa * atom_launches / step_s / 1e9
    traffic = None if traffic_bytes is None else traffic_bytes * launches / step_s / 1e9
    return {
        "value": atom_steps / wall,
        "trials_per_s": n / wall,
        "accepted_exchanges_per_s": acc / wall,
        "accepted": acc,
        "p_acc": acc / max(1, n),
        "p_acc_wilson95": [lo, hi],
        "insertions": n_ins, "insertions_accepted": n_ins_acc,
        "retried_trials": retried,
        "roofline": {
            "kernel": "k_step<1> (fused pair force + velocity Verlet)",
            "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "flop_per_atom_step": fpa,
            "traffic": traffic, "traffic_unit": "GB/s", "traffic_bytes_per_launch": traffic_bytes,
            "hbm": {"achieved": achieved_bytes, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved_bytes / HBM_PEAK_GBS, "bytes_per_atom_step": bpa},
            "mean_list_entries": mean_nbr,
            "avg_kernel_us": 1e3 * timing["step_ms"] / launches, "launches": timing["step_launches"],
            "timing": "HIP events around each step launch over the timing trials",
        },
        "rebuild_every": timing["rebuild_every"], "lanes_per_atom": timing["lanes"],
        "cell_cap": timing["cell_cap"], "list_cap": timing["nbr_cap"],
    }


def expected_acceptance(recs):
    """Mean Metropolis acceptance probability min(1, exp(ln R)) of the
    records: an estimator of the acceptance rate with far less variance
    than the count of accepted trials when acceptance is rare."""
    vals = []
    for r in recs:
        lr = r.ln_ratio
        vals.append(0.0 if (r.flags & 0x3) or not math.isfinite(lr) else math.exp(min(0.0, lr)))
    return sum(vals) / max(1, len(vals))


def jarzynski_beta_mu(dH, beta, volume, n_pairs):
    """Operating chemical potential of the current state: the beta mu at
    which the mean insertion ratio of Eq. (6), exp(-beta dH + beta mu + I),
    is 1 over the pilot insertions (I = 2 ln(V / (N + 1)), Lambda = 1)."""
    x = [-beta * d for d in dH if math.isfinite(d)]
    m = max(x)
    lme = m + math.log(sum(math.exp(v - m) for v in x) / len(x))
    return -2.0 * math.log(volume / (n_pairs + 1)) - lme


def choose_proposal(logits, bdH, c, ks=(4, 8, 16, 32, 64), scales=(0.25, 0.5, 1.0), margin=1.25,
                    draws=20000, seed=7):
    """(k, weight scale) of the learned proposal with the highest insertion
    acceptance, estimated from pilot insertions (out-of-fold network logit
    s_i and beta dH_i of sites drawn uniformly): each simulated move draws k
    pilot sites, picks one with probability proportional to
    exp(scale min(s, 10)) and takes min(1, exp(c - beta dH + ln(W/k) - log
    weight)), c = beta mu + I.  k stays at most an eighth of the pilot so
    that the resampled candidate sets do not repeat the same few sites.  The
    uniform proposal (scale 0) is kept unless the best pair beats it by the
    margin: rare acceptances make these estimates noisy."""
    import numpy as np
    if logits is None or len(logits) < 32:
        return 1, 0.0, {}
    rng = np.random.default_rng(seed)
    s = np.minimum(np.asarray(logits, dtype=np.float64), 10.0)
    bdH = np.asarray(bdH, dtype=np.float64)
    bdH = np.where(np.isfinite(bdH), bdH, np.inf)     # an overlap is never accepted
    m = len(s)
    est = {"uniform": float(np.mean(np.exp(np.minimum(0.0, c - bdH))))}
    best = (1, 0.0, est["uniform"] * margin)
    for k in ks:
        if 8 * k > m:
            continue
        idx = rng.integers(0, m, size=(draws, k))
        for scale in scales:
            lw = scale * s[idx]
            mx = lw.max(axis=1, keepdims=True)
            p = np.exp(lw - mx)
            lnWk = (mx[:, 0] + np.log(p.sum(axis=1))) - math.log(k)
            cum = np.cumsum(p, axis=1)
            u = rng.random(draws) * cum[:, -1]
            sel = np.minimum((cum < u[:, None]).sum(axis=1), k - 1)
            j = idx[np.arange(draws), sel]
            lnR = c - bdH[j] + lnWk - lw[np.arange(draws), sel]
            a = float(np.mean(np.exp(np.minimum(0.0, lnR))))
            est[f"k{k}_scale{scale}"] = a
            if a > best[2]:
                best = (k, scale, a)
    return best[0], best[1], est


def train_network(h4d, X, y, epochs, seed=1):
    """The proposal network trained on the GPU (FP32 forward, backward and
    Adam with decoupled weight decay; batch 128, lr 1e-3)."""
    net = h4d.Mlp(seed=seed)
    steps = max(50, (epochs * len(X)) // 128)
    losses = net.train(X, y, steps=steps, batch=128, lr=1e-3, seed=seed + 1, weight_decay=1e-2)
    return net, steps, losses


def out_of_fold(h4d, X, y, epochs, folds=5):
    """Logits of every pilot site from a network trained without it
    (folds-fold cross validation)."""
    import numpy as np
    oof = np.zeros(len(X))
    fold = np.arange(len(X)) % folds
    for f in range(folds):
        tr, te = fold != f, fold == f
        net, _, _ = train_network(h4d, X[tr], y[tr], epochs, seed=10 + f)
        oof[te] = net.forward(X[te])
        net.close()
    return oof


def proposal_ab(sys_, torch, h4d, arms, beta_mu, n_each, block=50):
    """Insertion and deletion acceptance of several proposals on one fixed
    state: forced moves at beta mu = -1000 (insertions) and +1000
    (deletions), which are never accepted, so the state does not change;
    each record's ln R is moved to the operating beta mu and the mean of
    min(1, R) taken.  The arms alternate in blocks so that they share the
    same state and device conditions.  arms: name -> (net, k, scale, bias
    (x_b, alpha_b) or None[, V_ex edge for early rejection])."""
    out = {name: {"ins": [], "del": [], "dM_ins": [], "dM_del": [], "s": 0.0, "n": 0, "instant": 0} for name in arms}
    done = 0
    while done < n_each:
        nb = min(block, n_each - done)
        for name, arm in arms.items():
            net, k, scale, bias = arm[:4]
            v_ex = arm[4] if len(arm) > 4 else 0.0
            sys_.set_bias(0.0, 0.0)
            sys_.set_early_rejection(0.0)
            if k > 0:
                sys_.set_proposal(net, k, 10.0, scale)
            else:
                sys_.set_proposal(None, 0)
            if bias is not None:
                sys_.set_bias(*bias)
            if v_ex > 0.0:
                sys_.set_early_rejection(v_ex)
            for move, bm, key in ((h4d.MOVE_INSERT, -1.0e3, "ins"), (h4d.MOVE_DELETE, 1.0e3, "del")):
                sys_.set_beta_mu(bm)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                arr = sys_.trials(nb, move, as_array=True)
                torch.cuda.synchronize()
                out[name]["s"] += time.perf_counter() - t0
                out[name]["n"] += nb
                shift = (beta_mu - bm) * (1.0 if move > 0 else -1.0)
                for q in range(nb):
                    r = arr[q]
                    ok = not (r.flags & 0x3) and math.isfinite(r.ln_ratio)
                    out[name][key].append(math.exp(min(0.0, r.ln_ratio + shift)) if ok else 0.0)
                    out[name]["dM_" + key].append(r.dM if ok else math.nan)
                    out[name]["instant"] += 1 if r.flags & 0x10 else 0
        done += nb
    sys_.set_proposal(None, 0)
    sys_.set_bias(0.0, 0.0)
    sys_.set_early_rejection(0.0)
    sys_.set_beta_mu(beta_mu)
    res = {}
    for name, o in out.items():
        p_ins = sum(o["ins"]) / max(1, len(o["ins"]))
        p_del = sum(o["del"]) / max(1, len(o["del"]))
        rate = o["n"] / max(1e-300, o["s"])
        res[name] = {"p_insert": p_ins, "p_delete": p_del, "trials_per_s": rate, "dM": (o["dM_ins"], o["dM_del"]),
                     "expected_exchanges_per_s": 0.5 * (p_ins + p_del) * rate,
                     "insertions": len(o["ins"]), "deletions": len(o["del"]),
                     "instant_share": o["instant"] / max(1, len(o["ins"]) + len(o["del"]))}
    if "uniform" in out and "learned" in out:
        res["gain"], res["gain_bootstrap90"] = ab_gain(out["uniform"], out["learned"])
    if "uniform" in out and "bimodal" in out:
        res["bimodal_gain"], res["bimodal_gain_bootstrap90"] = ab_gain(out["uniform"], out["bimodal"])
    if "bimodal" in out and "bimodal_early" in out:
        res["early_gain_over_bimodal"], res["early_gain_over_bimodal_bootstrap90"] = ab_gain(out["bimodal"],
                                                                                             out["bimodal_early"])
    return res


def ab_gain(u, l, reps=2000, seed=11):
    """Ratio of expected exchanges per second (another proposal over the
    uniform one) and its 90 % bootstrap interval (moves resampled within
    each arm and kind); None when the uniform arm's expected acceptance is
    below 1e-12 (the ratio is then meaningless)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    rate_u, rate_l = u["n"] / u["s"], l["n"] / l["s"]

    def ex(o, rate, pick):
        return 0.5 * (np.mean(pick(o["ins"])) + np.mean(pick(o["del"]))) * rate

    ident = np.asarray
    if ex(u, rate_u, ident) < 1e-12:       # the uniform arm's acceptance underflows: no ratio
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


def timed_trials(sys_, torch, n):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arr = sys_.trials(n, as_array=True)
    torch.cuda.synchronize()
    return [arr[q] for q in range(n)], time.perf_counter() - t0


# bimodal bias of the flying pair (x_b, alpha_b; Sec. II B 4): the paper's
# aqueous NaCl choice (4 A, 0.1 / A^2), and a contact-distance bias for the
# LJ ions (sigma = 1)
BIAS = {"lj32k": (1.0, 2.0), "water": (4.0, 0.1)}
# early rejection: edge of V_ex around the flying cation (LJ units; the water
# box leaves it out to keep its run short)
EARLY = {"lj32k": 1.2}

SINGLE = {
    "lj32k": ("config_lj_32k",
              "lj32k: 32,000 LJ ions, density 0.3, 200-step NEMD pair insert/delete, FP32 pair arithmetic / "
              "FP64 state, energies and work", "the 32,000-ion state",
              dict(n_atoms=32000, density=0.3, n_steps_per_trial=200, dt=0.005, w_max=2.5)),
    "water": ("config_water_nacl",
              "water: 8,000 rigid SPC/E waters + 150 NaCl pairs in a 62 A box, 298 K, 500-step NEMD NaCl-pair "
              "insert/delete (dt 1 fs, w_max 3 A, kappa_sr 1/A), FP32 pair arithmetic / FP64 state, energies "
              "and work", "the aqueous NaCl state",
              dict(n_atoms=24300, n_waters=8000, n_pairs=150, box_A=62.0, n_steps_per_trial=500, dt_fs=1.0,
                   w_max_A=3.0)),
}


def uniform_leg_speculative(args, h4d, torch, w, beta_mu):
    """The uniform chain run speculatively on args.replicas copies of its
    state (the records equal a one-by-one run of the same trials): timed
    trials, then timing trials with HIP events on the step kernel.  Returns
    (records, wall, timing, atom launches of the timing trials, info)."""
    spec = h4d.Speculative.from_workload(w, args.replicas, beta_mu=beta_mu)
    tuned = spec.autotune(2) if args.autotune else None
    if tuned:
        note(f"speculative autotune: {tuned[0]} lanes per atom, rebuild every {tuned[1]} steps")
    if args.warmup:
        spec.trials(args.warmup)
    r0 = spec.rounds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arr = spec.trials(args.steps, as_array=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rounds = spec.rounds - r0
    recs = [arr[q] for q in range(args.steps)]
    note(f"uniform, speculative: {args.steps} trials in {rounds} rounds of {args.replicas} replicas, {wall:.1f} s")
    spec.set_timing(True)
    r1 = spec.rounds
    tarr = spec.trials(args.timing_trials, as_array=True)
    timing = spec.timing()
    spec.set_timing(False)
    t_rounds = spec.rounds - r1
    spec.close()
    # every replica integrates its trial in every round
    n_mean = sum(tarr[q].n_atoms for q in range(args.timing_trials)) / max(1, args.timing_trials)
    nf = max(tarr[q].n_steps for q in range(args.timing_trials)) if args.timing_trials else 0
    atom_launches = t_rounds * args.replicas * n_mean * (nf + 1)
    info = {"mode": "speculative", "replicas": args.replicas, "rounds": rounds,
            "trials_per_round": args.steps / max(1, rounds),
            "note": "replicas of the state run the next trials side by side; the chain keeps them up to the "
                    "first accepted one (the records equal a one-by-one run); value counts the chain's "
                    "trials only"}
    return recs, wall, timing, atom_launches, info


def gcmd_leg(args, h4d, torch, w, beta_mu, tuned):
    """The grand-canonical cycle of Fig. 1: an equilibrium phase of
    args.n_eq steps (generalized hybrid MC with partial momentum refresh)
    and one exchange trial that carries the state's momenta with the
    symmetric two-end reversal, one cycle after another on one box."""
    over = dict(beta_mu=beta_mu, momenta=1, md_refresh=args.md_refresh)
    if tuned:
        over.update(lanes_per_atom=tuned[0], rebuild_every=tuned[1])
    g = h4d.System.from_workload(w, **over)
    g.md_phase(args.n_eq)
    g.trial()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    md_recs, tr_recs = [], []
    t_md = 0.0
    for _ in range(args.gcmd_cycles):
        t1 = time.perf_counter()
        md_recs.append(g.md_phase(args.n_eq)[0])
        torch.cuda.synchronize()
        t_md += time.perf_counter() - t1
        tr_recs.append(g.trial())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    n_md = sum(r["accepted"] for r in md_recs)
    n_tr = sum(r["accepted"] for r in tr_recs)
    steps = sum(r["n_atoms"] * (r["n_steps"] + 1) for r in md_recs + tr_recs)
    note(f"gcmd: {args.gcmd_cycles} cycles of {args.n_eq} equilibrium steps and one trial in {wall:.1f} s")
    carried = None
    if args.gcmd_trials > 0 and args.replicas > 1:
        # runs of trials with carried momenta from the same state: one after
        # another, and on speculative replicas (the same records when the
        # launch shape and rebuild interval are fixed)
        runs = {}
        for kind in ("one_by_one", "speculative"):
            h = (h4d.System.from_workload(w, **over) if kind == "one_by_one"
                 else h4d.Speculative.from_workload(w, args.replicas, **over))
            h.trials(4)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            recs = h.trials(args.gcmd_trials)
            torch.cuda.synchronize()
            runs[kind] = (recs, time.perf_counter() - t1, getattr(h, "rounds", None))
            h.close()
        (ra, wa, _), (rb, wb, rounds) = runs["one_by_one"], runs["speculative"]
        same = all(a == dict(b, n_rebuilds=a["n_rebuilds"]) for a, b in zip(ra, rb)) if tuned else None
        carried = {"trials": args.gcmd_trials, "replicas": args.replicas,
                   "one_by_one_trials_per_s": len(ra) / wa, "speculative_trials_per_s": len(rb) / wb,
                   "speedup": wa / max(wb, 1e-300), "accepted": sum(r["accepted"] for r in rb),
                   "records_equal": same}
        note(f"gcmd: {args.gcmd_trials} carried-momentum trials, one by one {wa:.1f} s, on {args.replicas} "
             f"replicas {wb:.1f} s, records equal: {same}")
    p_tr = n_tr / max(1, len(tr_recs))
    nf = tr_recs[0]["n_steps"] if tr_recs else 0
    return {
        "cycle": f"equilibrium phase of {args.n_eq} steps (partial momentum refresh c = {args.md_refresh}, "
                 "Metropolis on dH) + one trial with carried momenta and the two-end reversal",
        "cycles": args.gcmd_cycles, "wall_s": wall, "ms_per_cycle": 1e3 * wall / max(1, args.gcmd_cycles),
        "equilibrium_share_of_wall": t_md / max(wall, 1e-300),
        "atom_steps_per_s": steps / max(wall, 1e-300),
        "equilibrium_acceptance": n_md / max(1, len(md_recs)),
        "equilibrium_mean_abs_beta_dH": sum(abs(r["dH"]) for r in md_recs) / max(1, len(md_recs)) / w.params["kT"],
        "trials_accepted": n_tr, "trial_acceptance": p_tr,
        "efficiency_per_step": p_tr / max(1, nf + args.n_eq),
        "carried_momentum_trials": carried,
    }


def bench_single(args, h4d, W, torch):
    import numpy as np
    maker, desc, label, shape = SINGLE[args.workload]
    w = getattr(W, maker)()
    w.params.update(capacity=w.n + 1024)
    if args.rebuild_every:
        w.params.update(rebuild_every=args.rebuild_every)
    if args.lanes:
        w.params.update(lanes_per_atom=args.lanes)
    if args.skin > 0:
        w.params.update(skin=args.skin)
    speculative = args.replicas > 1
    sys_ = h4d.System.from_workload(w)
    tuned = sys_.autotune(4 if args.workload == "lj32k" else 2) if args.autotune else None
    if tuned:
        note(f"autotune: {tuned[0]} lanes per atom, rebuild every {tuned[1]} steps")
    if args.warmup:
        sys_.trials(args.warmup)
    # pilot: forced uniform insertions that are never accepted (beta mu far
    # below equilibrium), recording each site's features and dH
    sys_.set_beta_mu(-1.0e3)
    sys_.set_proposal(None, 1)
    feats, dH = [], []
    t0 = time.perf_counter()
    for _ in range(args.pilot):
        r = sys_.trial(h4d.MOVE_INSERT)
        feats.append(sys_.last_site_features())
        dH.append(r["dH"])
    pilot_s = time.perf_counter() - t0
    note(f"pilot: {args.pilot} insertions in {pilot_s:.1f} s")
    st = sys_.state()
    beta = 1.0 / w.params["kT"]
    L = w.params["box"][0]
    bmu_eq = jarzynski_beta_mu(dH, beta, L ** 3, st["nsalt"]) if dH else None
    if args.beta_mu is None and bmu_eq is None:
        raise SystemExit("bench.py: --pilot 0 needs --beta-mu")
    beta_mu = args.beta_mu if args.beta_mu is not None else bmu_eq
    c = beta_mu + 2.0 * math.log(L ** 3 / (st["nsalt"] + 1))
    # the network learns the clipped log insertion ratio c - beta dH of the
    # pilot sites (GPU, FP32); out-of-fold logits choose k and the scale
    # (no pilot, or one too small for cross validation, keeps the uniform
    # proposal)
    net = None
    k_sel, scale_sel, est, oof_corr, steps, train_s, losses = 1, 0.0, {}, None, 0, 0.0, np.zeros(1)
    if len(feats) > 0:
        X = np.array(feats, dtype=np.float32)
        bdH = beta * np.array(dH)
        ok = np.isfinite(bdH)
        X, bdH = X[ok], bdH[ok]
        y = np.clip(c - bdH, -100.0, 10.0).astype(np.float32)
        t0 = time.perf_counter()
        oof = out_of_fold(h4d, X, y, args.train_epochs) if len(X) >= 40 else None
        k_sel, scale_sel, est = choose_proposal(oof, bdH, c, ks=tuple(k for k in (4, 8, 16, 32, 64)
                                                                       if k <= args.candidates))
        net, steps, losses = train_network(h4d, X, y, args.train_epochs)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        oof_corr = float(np.corrcoef(oof, y)[0, 1]) if oof is not None and np.std(oof) > 0 else None
        note(f"network: out-of-fold correlation {oof_corr}, chose k = {k_sel}, scale = {scale_sel}")
    # uniform proposal, one trial after another on the single box (the
    # reference of the speculative leg; the timed leg itself when it is off)
    sys_.set_beta_mu(beta_mu)
    sys_.set_proposal(None, 0)
    seq_n = min(args.seq_steps, args.steps) if speculative else args.steps
    seq_recs, seq_wall = timed_trials(sys_, torch, seq_n)
    note(f"uniform, one by one: {seq_n} trials in {seq_wall:.1f} s")
    # the learned proposal from the state the uniform run reached (the plain
    # uniform proposal when the pilot favours no weighting)
    if scale_sel > 0.0:
        sys_.set_proposal(net, k_sel, 10.0, scale_sel)
    lrecs, lwall = timed_trials(sys_, torch, args.learned_steps)
    note(f"learned: {args.learned_steps} trials in {lwall:.1f} s")
    sys_.set_proposal(None, 0)
    # both proposals on the state the chains reached, alternating, with
    # forced moves that leave it unchanged
    arms = {"uniform": (None, 0, 0.0, None)}
    if scale_sel > 0.0:
        arms["learned"] = (net, k_sel, scale_sel, None)
    arms["bimodal"] = (None, 0, 0.0, BIAS[args.workload])
    if args.workload in EARLY:   # the bias with early rejection of pairs in contact
        arms["bimodal_early"] = (None, 0, 0.0, BIAS[args.workload], EARLY[args.workload])
    ab = proposal_ab(sys_, torch, h4d, arms, beta_mu, args.ab_trials) if args.ab_trials > 0 else None
    works = None
    if ab is not None:
        note(f"fixed-state comparison: {args.ab_trials} insertions and deletions per proposal")
        works = ab["uniform"]["dM"]
        for name in arms:
            ab[name].pop("dM")
    # step-kernel duration: further trials with HIP events around every
    # launch of the fused step kernel (on the library's stream)
    n_seq_timing = args.timing_trials if seq_n > 0 else 0
    sys_.set_timing(True)
    tarr = sys_.trials(n_seq_timing, as_array=True)
    seq_timing = sys_.timing()
    sys_.set_timing(False)
    sys_.close()
    if net is not None:
        net.close()
    gcmd = gcmd_leg(args, h4d, torch, w, beta_mu, tuned) if args.gcmd_cycles > 0 and not w.params["water"] else None
    traffic = counted_traffic(TRAFFIC_FILE) if args.workload == "lj32k" else None
    seq_timing_recs = [tarr[q] for q in range(n_seq_timing)]
    if speculative:
        recs, wall, timing, atom_launches, execution = uniform_leg_speculative(args, h4d, torch, w, beta_mu)
        out = summarize(recs, wall, timing, None, traffic, atom_launches=atom_launches)
        if seq_n > 0:
            seq = summarize(seq_recs, seq_wall, seq_timing, seq_timing_recs, None)
            out["sequential"] = {k: seq[k] for k in ("value", "trials_per_s", "accepted",
                                                     "accepted_exchanges_per_s", "p_acc", "rebuild_every",
                                                     "lanes_per_atom")}
            out["sequential"]["trials"] = seq_n
            out["sequential"]["expected_exchanges_per_s"] = expected_acceptance(seq_recs) * seq["trials_per_s"]
            out["sequential"]["roofline"] = {k: seq["roofline"][k] for k in ("achieved", "frac", "avg_kernel_us",
                                                                              "mean_list_entries")}
    else:
        recs, wall = seq_recs, seq_wall
        execution = {"mode": "one trial after another"}
        out = summarize(recs, wall, seq_timing, seq_timing_recs, traffic)
    out["execution"] = execution
    out["expected_acceptance"] = expected_acceptance(recs)
    out["expected_exchanges_per_s"] = out["expected_acceptance"] * out["trials_per_s"]
    l_acc = sum(r.accepted for r in lrecs)
    lo, hi = wilson(l_acc, len(lrecs))
    l_exp = expected_acceptance(lrecs)
    l_rate = len(lrecs) / max(lwall, 1e-300)
    seq_exp = expected_acceptance(seq_recs) * len(seq_recs) / max(seq_wall, 1e-300) if seq_recs else 0.0
    out["learned"] = {
        "proposal": (f"multiple-try, k = {k_sel} candidates weighted by exp({scale_sel} min(s, 10)), s the "
                     "trained network's logit (BF16 matrix-core inference)" if scale_sel > 0.0 else
                     "uniform: on the pilot's out-of-fold logits no (k, scale) beat it by the margin"),
        "execution": "one trial after another (single box)",
        "candidates": k_sel, "weight_scale": scale_sel,
        "choice_estimates": est,
        "value": sum(r.n_atoms * r.n_steps for r in lrecs) / max(lwall, 1e-300), "unit": "atom-steps/s",
        "trials": len(lrecs), "trials_per_s": l_rate,
        "accepted": l_acc, "accepted_exchanges_per_s": l_acc * l_rate / max(1, len(lrecs)),
        "p_acc": l_acc / max(1, len(lrecs)), "p_acc_wilson95": [lo, hi],
        "expected_acceptance": l_exp, "expected_exchanges_per_s": l_exp * l_rate,
        "gain_expected_exchanges_per_s_vs_one_by_one_uniform": l_exp * l_rate / max(1e-300, seq_exp),
        "pilot_insertions": args.pilot, "pilot_s": pilot_s, "train_steps": steps, "train_s": train_s,
        "train_loss_first": float(losses[:10].mean()), "train_loss_last": float(losses[-50:].mean()),
        "target": "clip(beta mu + I - beta dH, -100, 10)",
        "fixed_state_comparison": ab,
        "fixed_state_gain": ab.get("gain", 1.0 if scale_sel == 0.0 else None) if ab is not None else None,
        "fixed_state_gain_bootstrap90": ab.get("gain_bootstrap90") if ab is not None else None,
        "out_of_fold_corr_logit_vs_target": oof_corr,
    }
    if gcmd is not None:
        out["gcmd"] = gcmd
    out["bimodal_bias"] = {
        "x_b": BIAS[args.workload][0], "alpha_b": BIAS[args.workload][1],
        "note": "the paper's bias of the flying pair's separation (Sec. II B 4), in the fixed-state comparison",
        "fixed_state_gain": ab.get("bimodal_gain") if ab is not None else None,
        "fixed_state_gain_bootstrap90": ab.get("bimodal_gain_bootstrap90") if ab is not None else None,
    }
    if ab is not None and "bimodal_early" in ab:
        out["early_rejection"] = {
            "v_ex_edge": EARLY[args.workload],
            "note": "the bias with early rejection (pairs whose anion lies in the cube V_ex around the cation are "
                    "exchanged instantly, no trajectory), in the fixed-state comparison",
            "instant_share": ab["bimodal_early"]["instant_share"],
            "gain_over_bias_alone": ab.get("early_gain_over_bimodal"),
            "gain_over_bias_alone_bootstrap90": ab.get("early_gain_over_bimodal_bootstrap90"),
        }
    # the chemical potential and the predicted acceptance from the uniform
    # arm's work distributions (Crooks' theorem solved by BAR, Eq. 21)
    if works is not None:
        from paper_2307_11447_amd import analysis
        cal = analysis.work_summary(works[0], works[1], beta, beta_mu)
        cal["note"] = ("uniform forced insertions and deletions on one fixed state (no move accepted): "
                       "beta mu from BAR, P_acc predicted by Eq. (21) at the operating beta mu")
        cal["beta_mu_operating"] = beta_mu
        cal["observed_p_acc_uniform"] = (sum(r.accepted for r in recs) / len(recs)) if recs else None
        out["mu_calibration"] = cal
    config = dict({"workload": desc + "; value: uniform proposal" +
                   (f", {args.replicas} speculative replicas of the one chain" if speculative else "") +
                   "; 'learned': the trained multiple-try proposal from the same state"}, **shape)
    config.update({
        "beta_mu": beta_mu, "beta_mu_source": "given" if args.beta_mu is not None else
        "Jarzynski estimate from the pilot insertions (equilibrium operating point)",
        "beta_mu_jarzynski": bmu_eq,
        "skin": w.params["skin"], "proposal": "uniform", "parallelism": "single chain, one GPU",
    })
    base = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_steps, label)
    return out, config, base


def bench_batched(args, h4d, W, torch):
    ws = W.config_batched()
    for w in ws:
        w.params.update(beta_mu=args.beta_mu, rebuild_every=args.rebuild_every, lanes_per_atom=args.lanes)
        if args.skin > 0:
            w.params.update(skin=args.skin)
    bat = h4d.Batch.from_workloads(ws)
    tuned = bat.autotune(1) if args.autotune else None
    if tuned:
        note(f"autotune: {tuned[0]} lanes per atom, rebuild every {tuned[1]} steps")
    if args.warmup:
        bat.run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arr = bat.run(args.steps, as_array=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = [arr[q] for q in range(len(ws) * args.steps)]
    bat.set_timing(True)
    tarr = bat.run(args.timing_trials, as_array=True)
    timing = bat.timing()
    bat.set_timing(False)
    bat.close()
    out = summarize(recs, wall, timing, [tarr[q] for q in range(len(ws) * args.timing_trials)],
                    counted_traffic(TRAFFIC_FILE_BATCHED))
    config = {
        "workload": "batched256: 256 LJ-electrolyte boxes, N even in [1000, 16000] (2,220,126 ions), "
                    "density U[0.1, 0.4], N_f ~ U{100..400} per trial, FP32 pair arithmetic / FP64 state, "
                    "uniform proposal; every box runs its trial in one round of launches",
        "n_boxes": len(ws), "n_atoms": sum(w.n for w in ws), "trials_per_box": args.steps,
        "dt": 0.005, "w_max": 2.5, "beta_mu": args.beta_mu, "skin": ws[0].params["skin"],
        "proposal": "uniform", "parallelism": "256 boxes, one GPU",
    }
    big = max(ws, key=lambda w: w.n)
    base = None if args.no_cpu_baseline else cpu_baseline(big, args.cpu_steps,
                                                          f"the largest box ({big.n} ions)")
    return out, config, base


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("lj32k", "water", "batched"), default="lj32k")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed exchange trials (lj32k, default 2000) or trials per box (batched, default 20)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed trials first (default 20 / 2)")
    ap.add_argument("--beta-mu", type=float, default=None,
                    help="beta mu (default: lj32k, the Jarzynski estimate from the pilot; batched, -4)")
    ap.add_argument("--pilot", type=int, default=None,
                    help="single box: pilot insertions for the network (default 1200 / water 1000)")
    ap.add_argument("--train-epochs", type=int, default=30, help="single box: passes over the pilot data")
    ap.add_argument("--candidates", type=int, default=64,
                    help="single box: largest candidate count the learned proposal may choose")
    ap.add_argument("--learned-steps", type=int, default=None,
                    help="single box: timed learned trials (default: as many as --steps)")
    ap.add_argument("--replicas", type=int, default=8,
                    help="single box: speculative replicas of the chain for the timed uniform trials (<= 1: "
                         "one trial after another)")
    ap.add_argument("--seq-steps", type=int, default=None,
                    help="single box with replicas: one-by-one uniform trials timed for reference "
                         "(default 300 / water 60)")
    ap.add_argument("--ab-trials", type=int, default=None,
                    help="single box: forced insertions and deletions per proposal on the final state "
                         "(default 400)")
    ap.add_argument("--timing-trials", type=int, default=None,
                    help="trials run after the timed region with HIP events on the step kernel (20 / 2)")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle sample length (NEMD steps)")
    ap.add_argument("--gcmd-cycles", type=int, default=10,
                    help="single ion box: grand-canonical cycles (equilibrium phase + one trial) timed after the rest")
    ap.add_argument("--n-eq", type=int, default=1000, help="steps of an equilibrium phase (the paper's N_eq)")
    ap.add_argument("--gcmd-trials", type=int, default=200,
                    help="trials with carried momenta timed one by one and on speculative replicas (0: none)")
    ap.add_argument("--md-refresh", type=float, default=0.5, help="momentum persistence c of the equilibrium phase")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rebuild-every", type=int, default=0, help="list rebuild interval (0: library default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: library default)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library's lanes per atom and automatic rebuild interval instead of timing "
                         "the choices first")
    ap.add_argument("--skin", type=float, default=0.0, help="Verlet skin (0: workload default)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the stream-copy probe on MIB mebibytes and print its bandwidth")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "boxes are independent Markov chains and would shard across GPUs without communication, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    batched = args.workload == "batched"
    water = args.workload == "water"
    if args.steps is None:
        args.steps = 20 if batched else (400 if water else 2000)
    if args.warmup is None:
        args.warmup = 2 if batched else (5 if water else 20)
    if args.timing_trials is None:
        args.timing_trials = 2 if batched else (4 if water else 20)
    if args.learned_steps is None:
        args.learned_steps = args.steps
    if args.pilot is None:
        args.pilot = 1000 if water else 1200
    if args.ab_trials is None:
        args.ab_trials = 400
    if args.seq_steps is None:
        args.seq_steps = 60 if water else 300
    if batched and args.beta_mu is None:
        args.beta_mu = -4.0

    import torch
    from paper_2307_11447_amd import h4d
    from paper_2307_11447_amd import workloads as W

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        ms = h4d.stream_copy(nbytes, 20)
        print(json.dumps({"probe": "stream_copy", "bytes": nbytes, "ms": ms,
                          "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return

    out, config, base = (bench_batched if batched else bench_single)(args, h4d, W, torch)
    line = {
        "metric": METRIC,
        "value": out.pop("value"),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": config,
    }
    line["ms_per_step"] = 1e3 / out["trials_per_s"] * (config.get("n_boxes", 1))
    line.update(out)
    if base is not None:
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
