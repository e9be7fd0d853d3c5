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


def summarize(recs, wall, timing, timing_recs, traffic_bytes):
    """Throughput, acceptance and the step kernel's roofline from trial
    records (recs: the timed trials; timing_recs: the trials run with HIP
    events around every step launch)."""
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
    atom_launches = sum(r.n_atoms * (r.n_steps + 1) for r in timing_recs)
    step_s = timing["step_ms"] * 1e-3
    launches = max(1, timing["step_launches"])
    achieved = bpa * atom_launches / step_s / 1e9
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
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_bytes_per_launch": traffic_bytes,
            "bytes_per_atom_step": bpa, "mean_list_entries": mean_nbr,
            "avg_kernel_us": 1e3 * timing["step_ms"] / launches, "launches": timing["step_launches"],
            "timing": "HIP events around each step launch over the timing trials",
        },
        "rebuild_every": timing["rebuild_every"], "lanes_per_atom": timing["lanes"],
        "cell_cap": timing["cell_cap"], "list_cap": timing["nbr_cap"],
    }


def bench_single(args, h4d, W, torch):
    w = W.config_lj_32k()
    w.params.update(beta_mu=args.beta_mu, rebuild_every=args.rebuild_every, lanes_per_atom=args.lanes,
                    capacity=w.n + 1024)
    if args.skin > 0:
        w.params.update(skin=args.skin)
    sys_ = h4d.System.from_workload(w)
    if args.warmup:
        sys_.trials(args.warmup)
    # timed region: every trial launched as one captured HIP graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arr = sys_.trials(args.steps, as_array=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = [arr[q] for q in range(args.steps)]
    # step-kernel duration: the same trials continue with HIP events around
    # every launch of the fused step kernel (on the library's stream)
    sys_.set_timing(True)
    tarr = sys_.trials(args.timing_trials, as_array=True)
    timing = sys_.timing()
    sys_.set_timing(False)
    sys_.close()
    out = summarize(recs, wall, timing, [tarr[q] for q in range(args.timing_trials)],
                    counted_traffic(TRAFFIC_FILE))
    config = {
        "workload": "lj32k: 32,000 LJ ions, density 0.3, 200-step NEMD pair insert/delete, "
                    "FP32 pair arithmetic / FP64 state, energies and work, uniform proposal",
        "n_atoms": w.n, "density": 0.3, "n_steps_per_trial": 200, "dt": 0.005, "w_max": 2.5,
        "beta_mu": args.beta_mu, "skin": w.params["skin"], "proposal": "uniform",
        "parallelism": "single box, one GPU",
    }
    base = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_steps, "the 32,000-ion state")
    return out, config, base


def bench_batched(args, h4d, W, torch):
    ws = W.config_batched()
    for w in ws:
        w.params.update(beta_mu=args.beta_mu, rebuild_every=args.rebuild_every, lanes_per_atom=args.lanes)
        if args.skin > 0:
            w.params.update(skin=args.skin)
    bat = h4d.Batch.from_workloads(ws)
    if args.autotune:
        bat.autotune(1)
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
    ap.add_argument("--workload", choices=("lj32k", "batched"), default="lj32k")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed exchange trials (lj32k, default 2000) or trials per box (batched, default 20)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed trials first (default 20 / 2)")
    ap.add_argument("--beta-mu", type=float, default=-4.0)
    ap.add_argument("--timing-trials", type=int, default=None,
                    help="trials run after the timed region with HIP events on the step kernel (20 / 2)")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle sample length (NEMD steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rebuild-every", type=int, default=0, help="list rebuild interval (0: library default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: library default)")
    ap.add_argument("--autotune", action="store_true", help="batched: pick lanes per atom by timing first")
    ap.add_argument("--skin", type=float, default=0.0, help="Verlet skin (0: workload default)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the stream-copy probe on MIB mebibytes and print its bandwidth")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU (asked for {args.gpus} GPUs, WORLD_SIZE={world}); "
              "boxes are independent Markov chains and would shard across GPUs without communication, "
              "but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    batched = args.workload == "batched"
    if args.steps is None:
        args.steps = 20 if batched else 2000
    if args.warmup is None:
        args.warmup = 2 if batched else 20
    if args.timing_trials is None:
        args.timing_trials = 2 if batched else 20

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
