"""Checkpoint and resume: a handle created from a saved state and its
counters continues the chain with the records, states and running sums of
the uninterrupted run, bitwise (FP32 forces, carried momenta with
equilibrium phases, rigid water)."""
import os
import sys
import tempfile

import numpy as np
import pytest

from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def same(ra, rb, what):
    assert ra.keys() == rb.keys()
    for k in ra:
        a, b = ra[k], rb[k]
        assert a == b or (a != a and b != b), (what, k, a, b)


def same_state(sa, sb):
    assert sa["n"] == sb["n"] and sa["nsalt"] == sb["nsalt"]
    for k in ("x", "v", "type", "mol", "tag"):
        assert np.array_equal(sa[k], sb[k]), k


def run(g, plan):
    """plan: a sequence of "t" (one trial) and integers (a phase of that many
    steps); the records in order."""
    out = []
    for step in plan:
        out.append(g.trial() if step == "t" else g.md_phase(step)[0])
    return out


def through_file(ck):
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.npz")
        np.savez(path, **ck)
        with np.load(path) as f:          # no pickled objects in the file
            return {k: f[k] for k in f.files}


@pytest.mark.parametrize("case", ["fp32", "momenta", "water"])
def test_resumed_chain_equals_the_uninterrupted_run(case):
    if case == "fp32":
        w = W.lj_electrolyte(400, 0.1, 4301, n_steps=40, precision="fp32")
        w.params.update(beta_mu=10.0)
        before, after = ["t"] * 10, ["t"] * 10
    elif case == "momenta":
        w = W.lj_electrolyte(400, 0.1, 4302, n_steps=20, precision="fp64")
        w.params.update(beta_mu=10.0, momenta=1, md_refresh=0.5)
        before, after = [10, "t", 10, "t", "t"], [10, "t", "t", 10, "t"]
    else:
        w = W.water_nacl(n_water=300, n_pairs=10, L=21.0, m=7, seed=4303)
        w.params.update(precision="fp32")
        before, after = ["t"] * 4, ["t"] * 4
    say(f"case checkpoint {case}: {w.n} atoms, {len(before)} steps before, {len(after)} after")
    g = h4d.System.from_workload(w)
    pre = run(g, before)
    ck = through_file(g.checkpoint())
    raw = h4d.Checkpoint.from_buffer_copy(ck["checkpoint"].tobytes())
    ins = sum(1 for x in pre if x["move"] == 1 and x["accepted"])
    assert raw.next_tag == int(w.tag.max()) + 1 + 2 * ins
    assert raw.trial == sum(1 for x in before if x == "t")
    assert raw.md_phases == sum(1 for x in before if x != "t")
    ref = run(g, after)
    ref_state, ref_obs = g.state(), g.observables()
    g.close()
    r = h4d.System.resume(ck)
    got = run(r, after)
    for q, (a, b) in enumerate(zip(ref, got)):
        same(a, b, f"{case} step {q}")
    same_state(ref_state, r.state())
    same(ref_obs, r.observables(), f"{case} observables")
    say(f"   {sum(x['accepted'] for x in pre)} of {len(pre)} accepted before the checkpoint, "
        f"{sum(x['accepted'] for x in ref)} of {len(ref)} after")
    r.close()


def test_restore_rejects_a_mismatched_handle():
    w = W.lj_electrolyte(300, 0.1, 4304, n_steps=10, precision="fp64")
    g = h4d.System.from_workload(w)
    g.trials(2)
    ck = g.checkpoint()
    g.close()
    # another seed: the chain would not continue
    ckb = dict(ck)
    raw = h4d.Checkpoint.from_buffer_copy(ck["checkpoint"].tobytes())
    other = h4d.System(dict(w.params, seed=w.params["seed"] + 1), ck["x"], ck["type"], ck["mol"], ck["tag"],
                       int(ck["nsalt"]))
    with pytest.raises(h4d.H4DError) as e:
        h4d._check(h4d.lib().h4d_restore_checkpoint(other._h, raw, len(ck["x"]), None))
    assert e.value.code == h4d.H4D_EINVAL
    other.close()
    # a next tag that an atom of the state already holds
    raw.next_tag = int(ck["tag"].max())
    ckb["checkpoint"] = np.frombuffer(bytes(raw), np.uint8).copy()
    with pytest.raises(h4d.H4DError) as e:
        h4d.System.resume(ckb)
    assert e.value.code == h4d.H4D_EINVAL
    # checkpoints serve single chains, not batches
    bat = h4d.Batch.from_workloads([w, W.lj_electrolyte(300, 0.1, 4305, n_steps=10, precision="fp64")])
    with pytest.raises(h4d.H4DError) as e:
        h4d._check(h4d.lib().h4d_save_checkpoint(bat._h, h4d.Checkpoint()))
    assert e.value.code == h4d.H4D_EINVAL
    bat.close()


def test_checkpoint_moves_between_one_by_one_and_speculative_runs():
    say("case checkpoint across handle kinds: lj1000 fp32, 4 replicas, 3 x 12 trials")
    w = W.lj_electrolyte(1000, 0.3, 4306, n_steps=40, precision="fp32")
    w.params.update(beta_mu=-5.0, rebuild_every=10, lanes_per_atom=8, capacity=w.n + 256)
    T = 12
    seq = h4d.System.from_workload(w)
    first = seq.trials(T)
    ck = through_file(seq.checkpoint())
    ref = seq.trials(2 * T)
    ref_state = seq.state()
    seq.close()
    # one-by-one -> speculative
    sp = h4d.Speculative.resume(ck, 4)
    got = sp.trials(T)
    for a, b in zip(ref[:T], got):
        same(dict(a, n_rebuilds=0), dict(b, n_rebuilds=0), f"speculative trial {a['trial']}")
    # speculative -> one-by-one
    ck2 = through_file(sp.checkpoint())
    sp.close()
    r = h4d.System.resume(ck2)
    got2 = r.trials(T)
    for a, b in zip(ref[T:], got2):
        same(dict(a, n_rebuilds=0), dict(b, n_rebuilds=0), f"resumed trial {a['trial']}")
    same_state(dict(ref_state, v=0), dict(r.state(), v=0))
    acc = [sum(x["accepted"] for x in part) for part in (first, ref[:T], ref[T:])]
    say(f"   accepted {acc[0]}, {acc[1]}, {acc[2]} of {T} in the three parts")
    assert sum(acc[1:]) > 0
    r.close()


def test_batch_checkpoint_resumes_every_box_and_a_box_alone():
    say("case batch checkpoint: 3 LJ boxes fp64 with carried momenta, 4 + 4 trials per box")
    ws = [W.lj_electrolyte(n, 0.1, 4600 + n, n_steps=20, precision="fp64") for n in (340, 400, 460)]
    for w in ws:
        w.params.update(momenta=1, md_refresh=0.3, beta_mu=10.0, rebuild_every=5, lanes_per_atom=8)
    bat = h4d.Batch.from_workloads(ws)
    bat.run(4)
    cks = [through_file(c) for c in bat.checkpoint()]
    ref = bat.run(4)
    ref_states = [bat.box_state(b) for b in range(3)]
    bat.close()
    r = h4d.Batch.resume(cks)
    got = r.run(4)
    for b in range(3):
        for q in range(4):
            same(dict(ref[b][q], n_rebuilds=0), dict(got[b][q], n_rebuilds=0), f"box {b} trial {q}")
        same_state(ref_states[b], r.box_state(b))
    r.close()
    # box 1's record on its own: a single-box handle with the box's edges and stream
    one = h4d.System.resume(cks[1])
    alone = one.trials(4)
    for q in range(4):
        a, b = ref[1][q], alone[q]
        assert (a["move"], a["accepted"], a["trial"]) == (b["move"], b["accepted"], b["trial"]), q
        assert abs(a["dH"] - b["dH"]) < 1e-9 * max(1.0, abs(a["dH"])), q
    say(f"   {sum(x['accepted'] for row in ref for x in row)} of 12 accepted after the checkpoint")
    one.close()
