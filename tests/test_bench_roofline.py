"""The bench's arithmetic on made-up inputs (no GPU): the step kernel's
roofline against HBM with the algorithmic bytes 4 n_list + 36 of the pair
pass plus 120 of the integration, the FLOP fraction beside it, the
acceptance summary of trial records, and the choice of the learned
proposal's weight scale at many candidates."""
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


def test_scale_choice_at_many_candidates():
    """The multiple-try ratio keeps the uniform ratio's mean, so a weighting
    gains only where uniform ratios above 1 are cut off.  Here 1 % of the
    uniform insertion sites have ln R = 5 and the rest -30, and the logits
    name them: at scale 1 nearly every chosen site is a good one and its
    ratio is Z e^5 / e^5 = Z > 1, so the insertion acceptance rises from
    0.01 to about 1; deletions (ln R = 50) are accepted either way.  Zero
    logits leave every estimate at the uniform one, and logits unrelated to
    the work keep the uniform proposal."""
    rng = np.random.default_rng(3)
    good = rng.random(5000) < 0.01
    lr_ins = np.where(good, 5.0, -30.0)
    lr_del = np.full(1000, 50.0)
    s_del = np.zeros(1000)
    scale, est = bench.choose_scale(lr_ins, lr_ins, s_del, lr_del)
    assert est["uniform"]["p_ins"] == pytest.approx(np.mean(np.exp(np.minimum(0.0, lr_ins))))
    assert est["uniform"]["p_del"] == pytest.approx(1.0)
    assert est["scale1.0"]["p_ins"] > 0.99 and scale == 1.0
    _, est0 = bench.choose_scale(np.zeros(5000), lr_ins, s_del, lr_del)
    for key in ("scale0.5", "scale1.0"):
        assert est0[key]["p_ins"] == pytest.approx(est0["uniform"]["p_ins"])
    scale2, _ = bench.choose_scale(rng.normal(0.0, 4.0, size=5000), lr_ins, s_del, lr_del)
    assert scale2 == 0.0
