"""GPU parity of the learned proposal on many boxes at once: a batch of
independent boxes and speculative replicas of one chain.

Every box draws its own candidates from its own Philox stream and trial
index, scores them in one matrix-core pass over all boxes' candidates, and
takes its own multiple-try step (one block per box).  Checked:
* a FP64 batch, box by box, replayed through the oracle with the GPU's
  logits (the multiple-try form of Sec. II B 4, Eqs. 15-16, generalized to
  a learned weight): identical moves, chosen sites and decisions, ln q within
  1e-12, dH and the work within 1e-6 relative (floor 1 kT);
* speculative replicas with the learned proposal equal the one-by-one chain
  bitwise (FP32, the same launch shape);
* exactness in a batch: ideal reservoirs under a strongly biased network
  keep P(N) proportional to y^(2N) / (N!)^2 in every box.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as O
from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_fp64_batch_learned_replays_oracle_per_box():
    k, scale = 24, 1.0
    say(f"case learned batch fp64: 3 boxes (900-1200 ions), k = {k}, 5 rounds, replayed per box")
    specs = [(900, 0.3), (1200, 0.25), (1000, 0.35)]      # every box >= 3 list cells per edge
    ws = []
    for b, (n, rho) in enumerate(specs):
        w = W.lj_electrolyte(n, rho, 3100 + b, n_steps=40, precision="fp64")
        w.params.update(seed=3100, stream=b, beta_mu=6.0, kappa_sr=0.4, lanes_per_atom=8)
        ws.append(w)
    net = h4d.Mlp(seed=5)
    net.set_weights(mlp.random_theta(33, scale=2.0))
    bat = h4d.Batch.from_workloads(ws)
    bat.set_proposal(net, k, 10.0, scale)
    n_acc = n_cmp = 0
    worst_feat = 0.0
    for rnd in range(5):
        states = [bat.box_state(b) for b in range(len(ws))]
        recs = bat.run(1)
        for b, w in enumerate(ws):
            rg = recs[b][0]
            st = states[b]
            o = O.OracleSystem(w.params, st["x"], st["type"], st["mol"], st["tag"], st["nsalt"], cap=st["n"] + 8)
            sites, fg, lg = bat.last_candidates(k, box=b)
            seen = {}

            def replay(X):
                seen["X"] = X
                return lg.astype(np.float64)

            ro, _ = o.trial_learned(rg["trial"], k, replay, scale=scale)
            assert rg["move"] == ro["move"] and rg["flags"] & 3 == ro["flags"], (rnd, b, rg, ro)
            if ro["flags"] & 1:
                continue
            assert "X" in seen
            err = np.abs(fg - seen["X"]) / (1.0 + np.abs(seen["X"]))
            worst_feat = max(worst_feat, float(err.max()))
            assert rg["tag_c"] == ro["tag_c"] and rg["tag_a"] == ro["tag_a"]
            assert rg["ln_proposal"] == pytest.approx(ro["ln_proposal"], rel=1e-12, abs=1e-12)
            for key in ("dH", "W_prot", "E_switch", "H0"):
                assert abs(rg[key] - ro[key]) <= 1e-6 * max(1.0, abs(ro[key])), (rnd, b, key)
            assert rg["accepted"] == ro["accepted"], (rnd, b, rg, ro)
            n_acc += rg["accepted"]
            n_cmp += 1
            if ro["move"] > 0:   # the chosen candidate is where the ghosts flew in
                after = bat.box_state(b)
                if rg["accepted"]:
                    pos = {int(t): x for t, x in zip(after["tag"], after["x"])}
                    hit = np.isclose(sites[:, :3], pos[rg["tag_c"]]).all(axis=1)
                    assert hit.any()
    say(f"   {n_cmp} learned moves compared, {n_acc} accepted; worst candidate feature difference {worst_feat:.2e}")
    assert n_cmp >= 12 and worst_feat <= 2e-4
    bat.close()
    net.close()


@pytest.mark.parametrize("replicas", [4, 7])
def test_speculative_learned_chain_equals_one_by_one(replicas):
    k = 64
    say(f"case learned speculative lj1500 fp32, {replicas} replicas, k = {k}, 24 trials")
    w = W.lj_electrolyte(1500, 0.3, 4343, n_steps=40, precision="fp32")
    w.params.update(beta_mu=-2.0, rebuild_every=10, lanes_per_atom=8, capacity=w.n + 256)
    net = h4d.Mlp(seed=6)
    net.set_weights(mlp.random_theta(34, scale=1.5))
    T = 24
    seq = h4d.System.from_workload(w)
    seq.set_proposal(net, k, 10.0, 0.7)
    rs = seq.trials(T)
    spec = h4d.Speculative.from_workload(w, replicas)
    spec.set_proposal(net, k, 10.0, 0.7)
    rp = spec.trials(T)
    n_acc = sum(r["accepted"] for r in rs)
    say(f"   accepted {n_acc} of {T}; {spec.rounds} rounds")
    assert 0 < n_acc < T
    for t in range(T):
        assert rp[t]["ln_proposal"] != 0.0 or rp[t]["flags"] & 1
        assert rp[t] == dict(rs[t], n_rebuilds=rp[t]["n_rebuilds"]), t
    a, b = seq.state(), spec.state()
    assert np.array_equal(a["tag"], b["tag"]) and np.array_equal(a["x"], b["x"])
    seq.close()
    spec.close()
    net.close()


def test_ideal_reservoirs_keep_their_law_under_a_biased_batch_proposal():
    from test_gpu_learned import crafted_bias_theta
    from test_gpu_observables import ideal_moments
    say("case ideal reservoirs, batch of 4 with a biased learned proposal k = 8 (6000 trials per box)")
    y, L = 3.0, 5.0
    ws = []
    for b in range(4):
        w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1, seed=50)
        w.params.update(capacity=256, stream=b)
        ws.append(w)
    net = h4d.Mlp(seed=4)
    net.set_weights(crafted_bias_theta())
    bat = h4d.Batch.from_workloads(ws)
    bat.set_proposal(net, 8)
    ns = [[] for _ in ws]
    lnq = []
    for chunk in range(12):
        recs = bat.run(500)
        for b in range(len(ws)):
            for r in recs[b]:
                ns[b].append(r["n_salt_after"])
                if r["move"] > 0 and not r["flags"]:
                    lnq.append(r["ln_proposal"])
    m1, _, _ = ideal_moments(y)
    allns = np.concatenate([np.array(x[300:]) for x in ns]).astype(np.float64)
    from test_gpu_observables import batch_means_se
    se = batch_means_se(allns, nb=40)
    say(f"   <N> {allns.mean():.4f} (closed form {m1:.4f}, se {se:.4f}); ln q spread {np.std(lnq):.3f}")
    assert np.std(lnq) > 0.5            # the proposal really is biased
    assert abs(allns.mean() - m1) < 5 * se + 1e-3
    bat.close()
    net.close()
