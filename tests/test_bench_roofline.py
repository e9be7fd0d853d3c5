"""The bench's arithmetic on made-up inputs (no GPU): the step kernel's
roofline against HBM with the algorithmic bytes 4 n_list + 36 of the pair
pass plus 120 of the integration, the FLOP fraction beside it, the
acceptance summary of trial records, and the log-space acceptance and
gain of the fixed-state comparison; the committed counter summaries match
the kernel sources and the instantiation they name; the refusal of long
256-box runs; the per-launch-shape kernel summary."""
import math
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_of_a_known_launch():
    # 10 trials of 1000 atoms and 99 steps: every trial integrates its atoms
    # at 100 launches; 1000 launches take 2 ms in all
    atom_launches = 10 * 1000 * 100
    timing = {"mean_nbr": 100.0, "step_ms": 2.0, "step_launches": 1000, "atom_launches": float(atom_launches),
              "rebuild_every": 10, "lanes": 4, "cell_cap": 64, "nbr_cap": 256}
    r = bench.roofline(timing, 1.0e6, "k")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == pytest.approx(8000.0)
    assert r["bytes_per_atom_step"] == 4 * 100 + 36 + 120
    assert r["achieved"] == pytest.approx((4 * 100 + 156) * atom_launches / 2e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["flop"]["achieved"] == pytest.approx((46 * 100 + 18) * atom_launches / 2e-3 / 1e12)
    assert r["flop"]["frac"] == pytest.approx(r["flop"]["achieved"] / 157.3)
    assert r["traffic"] == pytest.approx(1.0e6 * 1000 / 2e-3 / 1e9)
    assert r["avg_kernel_us"] == pytest.approx(2.0)
    assert bench.roofline(timing, None, "k")["traffic"] is None


def test_arm_summary_counts_and_expected_acceptance():
    recs = [SimpleNamespace(n_atoms=100, n_steps=50, accepted=1 if t == 3 else 0, move=1 if t % 2 else -1,
                            flags=0, ln_ratio=(0.5 if t == 3 else -2.0), n_salt_before=10,
                            n_salt_after=11 if t >= 3 else 10) for t in range(8)]
    out = bench.arm_summary(recs, 2.0, rounds=3)
    assert out["atom_steps_per_s"] == pytest.approx(8 * 100 * 50 / 2.0)
    assert out["accepted"] == 1 and out["insertions"] == 4 and out["deletions"] == 4
    assert out["insertions_accepted"] == 1 and out["deletions_accepted"] == 0
    e_ins = (1.0 + 3 * math.exp(-2.0)) / 4
    assert out["expected_p_ins"] == pytest.approx(e_ins)
    assert out["expected_p_del"] == pytest.approx(math.exp(-2.0))
    assert out["n_salt_first"] == 10 and out["n_salt_last"] == 11 and out["rounds"] == 3


def test_log_space_acceptance_and_gain():
    """The fixed-state comparison averages min(1, R) in log space (an
    equilibrium beta mu with short flights underflows): zeros count, a
    tenfold acceptance at the same trial rate is a log10 gain of exactly 1,
    and an arm that accepts nothing has no ratio."""
    assert bench.log_mean_exp([0.0, -math.inf]) == pytest.approx(math.log(0.5))
    assert bench.log_mean_exp([-800.0, -802.0]) == pytest.approx(-800.0 + math.log((1 + math.exp(-2)) / 2))
    assert bench.log_mean_exp([-math.inf]) == -math.inf
    u = {"ins": [math.log(1e-30)] * 40, "del": [math.log(3e-31)] * 40, "n": 80, "s": 2.0}
    l = {"ins": [math.log(1e-29)] * 40, "del": [math.log(3e-30)] * 40, "n": 80, "s": 2.0}
    g, ci = bench.ab_log_gain(u, l)
    assert g == pytest.approx(1.0) and ci[0] == pytest.approx(1.0) and ci[1] == pytest.approx(1.0)
    none = {"ins": [-math.inf] * 4, "del": [-math.inf] * 4, "n": 8, "s": 1.0}
    assert bench.ab_log_gain(none, l) == (None, None)


def test_bench_line_is_strict_json():
    import json
    import math
    line = {"a": -math.inf, "b": [1.0, math.nan, {"c": math.inf}], "d": "x", "e": 2}
    out = json.dumps(bench.finite_json(line), allow_nan=False)
    assert json.loads(out) == {"a": None, "b": [1.0, None, {"c": None}], "d": "x", "e": 2}


def test_committed_counter_summaries_describe_the_current_kernels():
    # every traffic summary the bench reads was taken on the kernel sources as
    # they are, and names the instantiation (lanes per atom, list-load kind)
    # it measured; the bench finds each one for exactly that instantiation
    from paper_2307_11447_amd import rocprof_summary
    h = rocprof_summary.kernel_source_hash()
    for workload, files in bench.TRAFFIC_FILES.items():
        for path in files:
            kv = bench._summary_fields(path)
            assert kv["kernel_source_sha256"] == h, path
            lanes, nt = int(kv["lanes_per_atom"]), int(kv["nontemporal_lists"])
            timing = {"lanes": lanes, "nt_lists": nt}
            assert bench.counted_traffic(workload, timing) == float(kv["traffic_bytes_per_launch"]), path
            assert bench.counted_traffic(workload, {"lanes": lanes, "nt_lists": 1 - nt}) is None, path
    assert bench.counted_valu_busy("water", {"lanes": 8, "nt_lists": 1}) is not None


def test_long_runs_of_the_256_box_workload_are_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "batched", "--steps", "500",
                        "--no-cpu-baseline"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "at most 7 trials per box" in r.stderr, (r.returncode, r.stderr)


def test_rocprof_shapes_groups_a_kernel_by_launch_shape(tmp_path):
    import sqlite3
    from paper_2307_11447_amd import rocprof_summary
    path = str(tmp_path / "run_results.db")
    db = sqlite3.connect(path)
    db.execute("create table kernels(name text, grid_size int, duration int, start int, end int)")
    for g, du in [(1000, 5000), (1000, 7000), (2000, 100)]:
        db.execute("insert into kernels values (?, ?, ?, 0, 1)", ("void h4d::k_step<1, 8, false, true>", g, du))
    db.execute("insert into kernels values (?, ?, ?, 0, 1)", ("h4d::k_settle", 1000, 9))
    db.commit()
    rows = rocprof_summary.shapes(path, "k_step<1").splitlines()
    assert len(rows) == 3 and "grid_size" in rows[0]
    first = rows[1].split()
    assert first[-6:] == ["1000", "2", "0.012", "6.00", "5.00", "7.00"], rows
    assert rows[2].split()[-5] == "1"
