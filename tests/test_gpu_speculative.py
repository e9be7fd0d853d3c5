"""Speculative trials of one chain: replicas of the state run the next
trials side by side and keep them up to the first accepted one.  Every
random number is keyed by the trial index and a rejected trial leaves the
state unchanged, so the chain must equal a one-by-one run of the same
trials: here bitwise (FP32 pair pass, the same lanes per atom and rebuild
interval in both runs), record for record and in the final state."""
import sys

import numpy as np
import pytest

from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("replicas,beta_mu", [(6, -5.0), (3, 2.0)])
def test_speculative_chain_equals_sequential_run(replicas, beta_mu):
    say(f"case speculative lj1000 fp32, {replicas} replicas, beta mu {beta_mu}, 40 trials")
    w = W.lj_electrolyte(1000, 0.3, 4242, n_steps=40, precision="fp32")
    w.params.update(beta_mu=beta_mu, rebuild_every=10, lanes_per_atom=8, capacity=w.n + 256)
    T = 40
    seq = h4d.System.from_workload(w)
    rs = seq.trials(T)
    spec = h4d.Speculative.from_workload(w, replicas)
    rp = spec.trials(T)
    n_acc = sum(r["accepted"] for r in rs)
    say(f"   accepted {n_acc} of {T}; {spec.rounds} rounds of {replicas} replicas")
    assert 0 < n_acc < T and spec.rounds < T
    for t in range(T):
        assert rp[t]["trial"] == t
        assert rp[t] == dict(rs[t], n_rebuilds=rp[t]["n_rebuilds"]), t
    a, b = seq.state(), spec.state()
    assert a["n"] == b["n"] and a["nsalt"] == b["nsalt"]
    assert np.array_equal(a["tag"], b["tag"]) and np.array_equal(a["x"], b["x"])
    for box in range(replicas):   # every replica holds the chain's state
        assert np.array_equal(spec.box_state(box)["x"], a["x"])
    oa, ob = seq.observables(), spec.box_observables(0)
    for key in ("n_trials", "n_ins", "n_ins_acc", "n_del", "n_del_acc", "N_mean", "N2_mean"):
        assert oa[key] == ob[key], key
    # and it goes on from there: the next trials continue the same chain
    r2 = spec.trials(5)
    s2 = seq.trials(5)
    assert [r["trial"] for r in r2] == list(range(T, T + 5))
    for x, y in zip(r2, s2):
        assert x == dict(y, n_rebuilds=x["n_rebuilds"])
    seq.close()
    spec.close()


def test_speculative_fp64_chain_follows_the_oracle():
    say("case speculative lj500 fp64, 5 replicas, 16 trials against the oracle")
    from oracle import oracle as O
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0)
    spec = h4d.Speculative.from_workload(w, 5)
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    recs = spec.trials(16)
    n_acc = 0
    for t, rg in enumerate(recs):
        ro = o.trial(t)
        assert rg["trial"] == t and rg["move"] == ro["move"] and rg["flags"] & 3 == ro["flags"]
        if not ro["flags"]:
            for key in ("dH", "W_prot", "E_switch", "H0"):
                assert abs(rg[key] - ro[key]) <= 1e-6 * max(1.0, abs(ro[key])), (t, key)
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        n_acc += rg["accepted"]
    say(f"   accepted {n_acc} of 16 in {spec.rounds} rounds")
    st = spec.state()
    assert st["n"] == o.n and np.array_equal(st["tag"], o.tag[: o.n])
    spec.close()


def test_speculative_water_chain_equals_sequential_run():
    """Rigid SPC/E water with NaCl (1,300 waters, 34.2 A box): at beta mu =
    400 insertions are accepted and deletions are not, so rounds end early
    and the replicas take new states with their waters."""
    say("case speculative water fp32, 4 replicas, 12 trials")
    w = W.water_nacl(n_water=1300, n_pairs=20, L=34.2, m=12, seed=81)
    w.params.update(precision="fp32", n_steps=120, beta_mu=400.0, rebuild_every=6, lanes_per_atom=8,
                    capacity=w.n + 256)
    T = 12
    seq = h4d.System.from_workload(w)
    rs = seq.trials(T)
    spec = h4d.Speculative.from_workload(w, 4)
    rp = spec.trials(T)
    n_acc = sum(r["accepted"] for r in rs)
    say(f"   accepted {n_acc} of {T}; {spec.rounds} rounds")
    for t in range(T):
        assert rp[t] == dict(rs[t], n_rebuilds=rp[t]["n_rebuilds"]), t
    assert 0 < n_acc < T, [(r["move"], r["flags"], r["dH"], r["ln_ratio"]) for r in rs]
    a, b = seq.state(), spec.state()
    assert a["n"] == b["n"] and np.array_equal(a["tag"], b["tag"]) and np.array_equal(a["x"], b["x"])
    for box in range(4):
        assert np.array_equal(spec.box_state(box)["x"], a["x"])
    seq.close()
    spec.close()
