"""GPU parity of the batched engine: independent boxes of uneven size and
density, each with its own N_f per trial, run together in one round of
launches.

* FP64: every box's trial sequence equals the oracle's run of that box
  alone (same seed, stream + b): identical moves and decisions, dH, W_prot
  and E_switch within 1e-6 relative (floor 1 kT).
* FP32: box b of a batch is bitwise identical to a single-box system
  created with box b's edges and stream (no cross-talk between boxes).
* Full size (256 boxes, about 2.2 million ions): the oracle recomputes the
  starting Hamiltonian of sampled boxes; rejected trials leave their box
  bitwise unchanged.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_boxes(prec, n_steps_min, n_steps_max, seed=2001):
    specs = [(600, 0.2), (900, 0.3), (1200, 0.35), (700, 0.25)]
    ws = []
    for b, (n, rho) in enumerate(specs):
        w = W.lj_electrolyte(n, rho, seed + b, precision=prec)
        w.params.update(n_steps=0, n_steps_min=n_steps_min, n_steps_max=n_steps_max,
                        seed=seed, stream=b, beta_mu=6.0, lanes_per_atom=8)
        ws.append(w)
    return ws


def rel_close(a, b, tol, floor=1.0):
    return abs(a - b) <= tol * max(abs(b), floor)


def test_fp64_batch_matches_oracle_per_box():
    say("case batch fp64: 4 boxes (600-1200 ions), N_f ~ U{20..40}, 8 trials per box")
    ws = small_boxes("fp64", 20, 40)
    bat = h4d.Batch.from_workloads(ws)
    assert bat.n_boxes == 4
    recs = bat.run(8)
    for b, w in enumerate(ws):
        o = O.OracleSystem.from_workload(w, cap=w.n + 64)
        for t in range(8):
            rg, ro = recs[b][t], o.trial(t)
            assert rg["trial"] == t and rg["move"] == ro["move"] and rg["n_steps"] == ro["n_steps"]
            assert rg["flags"] & 3 == ro["flags"]
            if not ro["flags"]:
                for key in ("dH", "W_prot", "E_switch", "H0", "H1"):
                    assert rel_close(rg[key], ro[key], 1e-6), (b, t, key, rg[key], ro[key])
            assert rg["accepted"] == ro["accepted"], (b, t, rg, ro)
        st = bat.box_state(b)
        assert st["n"] == o.n and np.array_equal(st["tag"], o.tag[: o.n])
        L = w.params["box"][0]
        d = st["x"] - o.x[: o.n]
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-8
        say(f"   box {b}: n {st['n']}, accepted {sum(r['accepted'] for r in recs[b])} of 8")
    bat.close()


def test_fp32_batch_box_equals_single_system_bitwise():
    say("case batch fp32: each box bitwise equal to its single-box run")
    ws = small_boxes("fp32", 30, 60, seed=2101)
    for w in ws:
        w.params.update(rebuild_every=10)   # the same rebuild schedule in both runs
    bat = h4d.Batch.from_workloads(ws)
    recs = bat.run(5)
    for b, w in enumerate(ws):
        single = h4d.System.from_workload(w)
        rs = single.trials(5)
        for t in range(5):
            assert recs[b][t] == dict(rs[t], n_rebuilds=recs[b][t]["n_rebuilds"]), (b, t)
        assert np.array_equal(bat.box_state(b)["x"], single.state()["x"])
        single.close()
    obs = bat.box_observables(2)
    assert obs["n_trials"] == 5 and obs["n_atoms"] == bat.box_state(2)["n"]
    bat.close()


def test_batch_full_size_start_hamiltonians():
    say("case batch full size: 256 boxes, N in [1000, 16000], density 0.1-0.4 (1 trial per box)")
    ws = W.config_batched()
    total = sum(w.n for w in ws)
    bat = h4d.Batch.from_workloads(ws)
    before = {b: bat.box_state(b) for b in (0, 77, 254)}
    recs = bat.run(1)
    say(f"   {total} ions; accepted {sum(r[0]['accepted'] for r in recs)} of 256")
    for b in (0, 77, 254):
        w, st = ws[b], before[b]
        o = O.OracleSystem(dict(w.params, stream=b), st["x"], st["type"], st["mol"], st["tag"], st["nsalt"],
                           cap=st["n"] + 8)
        ref = o.trial_begin(0)
        r = recs[b][0]
        say(f"   box {b}: n {st['n']} move {r['move']:+d} N_f {r['n_steps']} H0 {r['H0']:.6f} (oracle {ref['H0']:.6f})")
        assert r["move"] == ref["move"] and r["n_steps"] == ref["nf"]
        assert r["tag_c"] == ref["tag_c"] and r["tag_a"] == ref["tag_a"]
        assert r["H0"] == pytest.approx(ref["H0"], rel=1e-11)
        if r["move"] > 0:
            assert r["E_switch"] == pytest.approx(ref["E_switch"], rel=1e-9, abs=1e-9)
        assert math.isfinite(r["dH"])
        after = bat.box_state(b)
        if not r["accepted"]:
            assert np.array_equal(after["x"], st["x"])
    assert all(100 <= r[0]["n_steps"] <= 400 for r in recs)
    bat.close()
