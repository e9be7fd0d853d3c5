"""Equilibrium phases between trials and trials with carried momenta on
the GPU against the FP64 oracle (records, positions and momenta after every
step of a mixed sequence), in one box and in a batch."""
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


def close_state(g, o, atol=1e-7):
    assert g["n"] == o.n and g["nsalt"] == o.nsalt
    assert np.array_equal(g["tag"], o.tag[: o.n])
    L = o.pd["box"][0]
    d = g["x"] - o.positions()
    d -= L * np.round(d / L)
    assert np.abs(d).max() < atol
    assert np.abs(g["v"] - o.velocities()).max() < atol


def same_record(rg, ro, what):
    assert rg["move"] == ro["move"] and rg["accepted"] == ro["accepted"], (what, rg, ro)
    assert rg["trial"] == ro["trial"], what
    if not ro["flags"]:
        assert abs(rg["dH"] - ro["dH"]) < 1e-6 * max(1.0, abs(ro["dH"])), (what, rg["dH"], ro["dH"])
        assert rg["ln_u"] == pytest.approx(ro["ln_u"], abs=1e-12), what


@pytest.mark.parametrize("refresh,dt", [(0.0, 0.005), (0.6, 0.02)])
def test_md_phases_match_the_oracle(refresh, dt):
    say(f"case md phases lj300 fp64, refresh {refresh}, dt {dt}")
    w = W.lj_electrolyte(300, 0.3, 77, n_steps=20, precision="fp64")
    w.params.update(md_refresh=refresh, dt=dt)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    close_state(g.state(), o)             # the same initial momenta
    acc = 0
    for p in range(6):
        rg = g.md_phase(15)[0]
        ro = o.md_phase(p, 15)
        same_record(rg, ro, f"phase {p}")
        close_state(g.state(), o)
        acc += ro["accepted"]
    say(f"   accepted {acc} of 6")
    g.close()


def test_carried_momenta_sequence_matches_the_oracle():
    say("case carried momenta lj300 fp64: phases and trials interleaved")
    w = W.lj_electrolyte(300, 0.1, 78, n_steps=30, precision="fp64")
    w.params.update(momenta=1, md_refresh=0.5, beta_mu=10.0, kappa_sr=0.4)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    n_acc = 0
    for t in range(10):
        rg = g.md_phase(10)[0]
        ro = o.md_phase(t, 10)
        same_record(rg, ro, f"phase {t}")
        rg = g.trial()
        ro = o.trial(t)
        same_record(rg, ro, f"trial {t}")
        n_acc += ro["accepted"]
        close_state(g.state(), o, atol=1e-6)
    say(f"   trials accepted {n_acc} of 10")
    assert n_acc > 0
    g.close()


def test_batched_phases_match_the_oracle_per_box():
    say("case md phases, batch of 3 lj boxes fp64")
    ws = [W.lj_electrolyte(n, 0.1, 90 + n, n_steps=20, precision="fp64") for n in (340, 400, 460)]
    for w in ws:
        w.params.update(md_refresh=0.3, momenta=1, beta_mu=10.0)
    bat = h4d.Batch.from_workloads(ws)
    os_ = []
    for b, w in enumerate(ws):
        p = dict(ws[0].params, box=w.params["box"], stream=ws[0].params["stream"] + b)
        os_.append(O.OracleSystem(p, w.x, w.type, w.mol, w.tag, w.nsalt, cap=w.n + 64))
    n_acc = 0
    for t in range(4):
        rg = bat.md_phase(12)
        for b in range(3):
            same_record(rg[b], os_[b].md_phase(t, 12), f"box {b} phase {t}")
        rt = bat.run(1)
        for b in range(3):
            ro = os_[b].trial(t)
            same_record(rt[b][0], ro, f"box {b} trial {t}")
            n_acc += ro["accepted"]
    say(f"   trials accepted {n_acc} of 12")
    for b in range(3):
        close_state(bat.box_state(b), os_[b], atol=1e-6)
    bat.close()


def test_phase_on_speculative_replicas_keeps_them_equal():
    say("case md phase on 4 speculative replicas of lj300 fp64")
    w = W.lj_electrolyte(300, 0.1, 81, n_steps=20, precision="fp64")
    w.params.update(md_refresh=0.4, beta_mu=10.0)
    sp = h4d.Speculative.from_workload(w, 4)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    recs = sp.md_phase(12)
    ro = o.md_phase(0, 12)
    for r in recs:   # every replica ran the same phase
        same_record(r, ro, "phase 0")
    s0 = sp.box_state(0)
    close_state(s0, o)
    for b in range(1, 4):
        sb = sp.box_state(b)
        assert np.array_equal(sb["x"], s0["x"]) and np.array_equal(sb["v"], s0["v"])
    # the chain's trials go on from the phase's state
    rt = sp.trials(6)
    for t, rg in enumerate(rt):
        same_record(rg, o.trial(t), f"trial {t}")
    sp.close()


def test_phase_refuses_an_empty_trajectory():
    # (rigid water runs phases too: tests/test_gpu_water_md.py)
    w = W.lj_electrolyte(300, 0.3, 77, n_steps=20, precision="fp64")
    g = h4d.System.from_workload(w)
    with pytest.raises(h4d.H4DError) as e:
        g.md_phase(0)
    assert e.value.code == h4d.H4D_EINVAL
    g.close()


def _run_plan(g, plan, speculative):
    out = []
    for step in plan:
        if step == "md":
            out.append(g.md_phase(10)[0])
        else:
            out.extend(g.trials(step))
    return out


@pytest.mark.parametrize("case", ["salt_bm10", "salt_bm2", "empty_ideal_gas"])
def test_speculative_replicas_carry_momenta_like_one_by_one(case):
    if case.startswith("salt"):
        w = W.lj_electrolyte(400, 0.1, 4501, n_steps=20, precision="fp32")
        w.params.update(beta_mu=10.0 if case == "salt_bm10" else 2.0, momenta=1, md_refresh=0.5,
                        rebuild_every=10, lanes_per_atom=8, capacity=w.n + 256)
        plan = ["md", 8, "md", 8, 8]
    else:   # starts with no salt: rounds run one replica until an insertion is accepted
        w = W.ideal_gas(L=6.0, beta_mu=0.0, n_steps=3)
        w.params.update(momenta=1, md_refresh=0.5)
        plan = [30, 10]
    say(f"case carried momenta on 4 speculative replicas: {case}")
    seq = h4d.System.from_workload(w)
    sp = h4d.Speculative.from_workload(w, 4)
    ra = _run_plan(seq, plan, False)
    rb = _run_plan(sp, plan, True)
    for q, (a, b) in enumerate(zip(ra, rb)):
        assert a == dict(b, n_rebuilds=a["n_rebuilds"]), (q, a, b)
    sa = seq.state()
    for box in range(4):
        sb = sp.box_state(box)
        assert sa["n"] == sb["n"] and np.array_equal(sa["tag"], sb["tag"])
        assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["v"], sb["v"]), box
    acc = sum(r["accepted"] for r in ra if r["move"] != h4d.MOVE_MD)
    n_tr = sum(1 for r in ra if r["move"] != h4d.MOVE_MD)
    say(f"   {acc} of {n_tr} trials accepted; {sp.rounds} speculative rounds")
    assert 0 < acc < n_tr
    seq.close()
    sp.close()
