"""The bench's roofline arithmetic on made-up timings (no GPU): the step
kernel is priced against the vector FP32 rate with its algorithmic
operation count, and against HBM with its algorithmic bytes."""
import os
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_of_a_known_launch():
    # 10 trials of 1000 atoms and 99 steps: every trial integrates its atoms
    # at 100 launches; 1000 launches take 2 ms in all
    recs = [SimpleNamespace(n_atoms=1000, n_steps=99, accepted=t % 2, move=1 - 2 * (t % 2), flags=0)
            for t in range(10)]
    timing = {"mean_nbr": 100.0, "step_ms": 2.0, "step_launches": 1000, "rebuild_every": 10, "lanes": 4,
              "cell_cap": 64, "nbr_cap": 256}
    out = bench.summarize(recs, 1.0, timing, recs, traffic_bytes=1.0e6)
    r = out["roofline"]
    atom_launches = 10 * 1000 * 100
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == pytest.approx(157.3)
    flop = (46 * 100 + 18) * atom_launches
    assert r["flop_per_atom_step"] == 46 * 100 + 18
    assert r["achieved"] == pytest.approx(flop / 2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["hbm"]["achieved"] == pytest.approx((4 * 100 + 184) * atom_launches / 2e-3 / 1e9)
    assert r["hbm"]["frac"] == pytest.approx(r["hbm"]["achieved"] / 8000.0)
    assert r["traffic"] == pytest.approx(1.0e6 * 1000 / 2e-3 / 1e9) and r["traffic_unit"] == "GB/s"
    assert r["avg_kernel_us"] == pytest.approx(2.0)
    assert out["value"] == pytest.approx(10 * 1000 * 99)
