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


def counted_traffic():
    """HBM bytes per step launch from the committed rocprofv3 counter summary,
    or None if it is missing or was taken on different kernel sources."""
    from paper_2307_11447_amd import rocprof_summary
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
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


def cpu_baseline(w, n_steps):
    """The FP64 oracle, single threaded, on a bounded sample: one trial of
    the same 32,000-ion state with the trajectory cut to n_steps steps."""
    from oracle import build as ob
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        ob.build()
    params = dict(w.params, n_steps=n_steps)
    o = O.OracleSystem(params, w.x, w.type, w.mol, w.tag, w.nsalt, cap=w.n + 8)
    t0 = time.perf_counter()
    rec = o.trial(0)
    dt = time.perf_counter() - t0
    atoms = w.n
    return {"value": atoms * n_steps / dt, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 trial (move {rec['move']:+d}) of the 32,000-ion state with N_f cut to "
                      f"{n_steps} steps ({atoms * n_steps:.3g} atom-steps, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed exchange trials")
    ap.add_argument("--warmup", type=int, default=20, help="untimed trials first")
    ap.add_argument("--beta-mu", type=float, default=-4.0)
    ap.add_argument("--timing-trials", type=int, default=20,
                    help="trials run after the timed region with HIP events on the step kernel")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle sample length (NEMD steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rebuild-every", type=int, default=0, help="list rebuild interval (0: library default)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per atom (0: library default)")
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

    import torch
    from paper_2307_11447_amd import h4d
    from paper_2307_11447_amd import workloads as W

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        ms = h4d.stream_copy(nbytes, 20)
        print(json.dumps({"probe": "stream_copy", "bytes": nbytes, "ms": ms,
                          "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return

    w = W.config_lj_32k()
    w.params.update(beta_mu=args.beta_mu, rebuild_every=args.rebuild_every, lanes_per_atom=args.lanes)
    if args.skin > 0:
        w.params.update(skin=args.skin)
    sys_ = h4d.System.from_workload(w)
    if args.warmup:
        sys_.trials(args.warmup)
    # timed region: every trial launched as one captured HIP graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = sys_.trials(args.steps, as_array=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    # step-kernel duration: the same trials continue with HIP events around
    # every launch of the fused step kernel (on the library's stream)
    sys_.set_timing(True)
    sys_.trials(args.timing_trials)
    timing = sys_.timing()
    sys_.set_timing(False)
    n = args.steps
    atom_steps = sum(recs[q].n_atoms * recs[q].n_steps for q in range(n))
    acc = sum(recs[q].accepted for q in range(n))
    n_ins = sum(1 for q in range(n) if recs[q].move > 0)
    n_ins_acc = sum(recs[q].accepted for q in range(n) if recs[q].move > 0)
    retried = sum(1 for q in range(n) if recs[q].flags & h4d.FLAG_RETRIED)
    lo, hi = wilson(acc, n)
    mean_nbr = timing["mean_nbr"]
    n_atoms_mean = atom_steps / max(1, sum(recs[q].n_steps for q in range(n)))
    # algorithmic bytes of one fused step launch, per atom: 4 B per list
    # entry, 4 B list length, 16 B own fixed-point record, 32 B own FP64
    # position, 16 B fixed-point position at the list build, 64 B velocity in
    # and out, 48 B new position (FP64 + fixed point); neighbour records are
    # gathered through the caches and not counted
    bytes_per_atom = 4.0 * mean_nbr + 184.0
    avg_ms = timing["step_ms"] / max(1, timing["step_launches"])
    achieved = bytes_per_atom * n_atoms_mean / (avg_ms * 1e-3) / 1e9
    tb = counted_traffic()
    traffic = None if tb is None else tb / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": atom_steps / wall,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": n,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / n,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "lj32k: 32,000 LJ ions, density 0.3, 200-step NEMD pair insert/delete, "
                        "FP32 pair arithmetic / FP64 state, energies and work, uniform proposal",
            "n_atoms": w.n, "density": 0.3, "n_steps_per_trial": 200, "dt": 0.005, "w_max": 2.5,
            "beta_mu": args.beta_mu, "skin": w.params["skin"], "proposal": "uniform",
            "parallelism": "single box, one GPU",
        },
        "trials_per_s": n / wall,
        "accepted_exchanges_per_s": acc / wall,
        "accepted": acc,
        "p_acc": acc / n,
        "p_acc_wilson95": [lo, hi],
        "insertions": n_ins, "insertions_accepted": n_ins_acc,
        "roofline": {
            "kernel": "k_step<1> (fused pair force + velocity Verlet)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_bytes_per_launch": tb,
            "bytes_per_atom_step": bytes_per_atom, "mean_list_entries": mean_nbr,
            "avg_kernel_us": avg_ms * 1e3, "launches": timing["step_launches"],
            "timing": "HIP events around each step launch over the timing trials",
        },
        "rebuild_every": timing["rebuild_every"], "lanes_per_atom": timing["lanes"],
        "cell_cap": timing["cell_cap"], "list_cap": timing["nbr_cap"],
        "retried_trials": retried,
    }
    sys_.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
