"""Failure handling forced from the host: a full box refuses an insertion
with H4D_ECAPACITY and keeps its state and trial index, and a state whose
local density is twice the box average (a slab) outgrows the initial list
capacities, which grow, and still follows the oracle."""
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


def same_record(rg, ro, what):
    assert rg["move"] == ro["move"] and rg["accepted"] == ro["accepted"], (what, rg, ro)
    assert rg["trial"] == ro["trial"], what
    if not ro["flags"]:
        assert abs(rg["dH"] - ro["dH"]) < 1e-6 * max(1.0, abs(ro["dH"])), (what, rg["dH"], ro["dH"])


def test_full_box_refuses_an_insertion_and_keeps_its_state():
    say("case capacity: 510 LJ ions in a box of capacity 512, fp64")
    w = W.lj_electrolyte(510, 0.1, 4401, n_steps=20, precision="fp64")
    w.params.update(beta_mu=10.0, capacity=512)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    t = 0
    while True:   # insertions until one fills the box
        rg = g.trial(h4d.MOVE_INSERT)
        same_record(rg, o.trial(t, force_move=1), f"insertion {t}")
        t += 1
        if rg["accepted"]:
            break
        assert t < 10
    s0, n_trials = g.state(), g.observables()["n_trials"]
    assert s0["n"] == 512
    with pytest.raises(h4d.H4DError) as e:
        g.trial(h4d.MOVE_INSERT)
    assert e.value.code == h4d.H4D_ECAPACITY
    s1 = g.state()
    assert s1["n"] == s0["n"] and s1["nsalt"] == s0["nsalt"]
    for k in ("x", "type", "tag"):
        assert np.array_equal(s0[k], s1[k]), k
    assert g.observables()["n_trials"] == n_trials
    # the refused trial used no index: the deletions take it and the next ones
    g.set_beta_mu(-10.0)
    o.p.beta_mu = -10.0
    deleted = 0
    for q in range(4):
        rg = g.trial(h4d.MOVE_DELETE)
        same_record(rg, o.trial(t, force_move=-1), f"deletion {t}")
        deleted += rg["accepted"]
        t += 1
    say(f"   box filled at trial {t - 5}, {deleted} of 4 deletions accepted after the refusal")
    assert deleted > 0
    same_record(g.trial(h4d.MOVE_INSERT), o.trial(t, force_move=1), "insertion after the deletions")
    g.close()


def test_slab_state_grows_the_lists_and_follows_the_oracle():
    say("case slab: 1000 LJ ions at density 0.4 in a box twice as long in x, fp64")
    w = W.lj_electrolyte(1000, 0.4, 4402, n_steps=20, precision="fp64")
    L = w.params["box"][0]
    w.params["box"] = [2.0 * L, L, L]
    w.params.update(beta_mu=4.0)
    assert w.x[:, 0].max() < L
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    for t in range(6):
        same_record(g.trial(), o.trial(t), f"trial {t}")
    tm = g.timing()
    say(f"   list capacity {tm['nbr_cap']} per atom, cell capacity {tm['cell_cap']}")
    st = g.state()
    d = st["x"] - o.positions()
    box = np.array(w.params["box"])
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-7
    g.close()
