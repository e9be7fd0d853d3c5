"""Early rejection on the GPU against the FP64 oracle: a pair whose anion
lies in the cube V_ex around the flying cation is exchanged instantly (no
trajectory); every record, instant or not, matches the oracle's."""
import sys

import pytest

from oracle import oracle as O
from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["params", "setter", "speculative"])
def test_early_rejection_trials_match_oracle(mode):
    say(f"case early rejection lj300 fp64, V_ex edge 7, 40 trials, {mode}")
    w = W.lj_electrolyte(300, 0.1, 79, n_steps=20, precision="fp64")
    w.params.update(v_ex_edge=7.0, beta_mu=10.0)
    if mode == "speculative":
        g = h4d.Speculative.from_workload(w, 4)
        recs = g.trials(40)
    elif mode == "setter":
        g = h4d.System.from_workload(w, v_ex_edge=0.0)
        g.set_early_rejection(7.0)
        recs = [g.trial() for _ in range(40)]
    else:
        g = h4d.System.from_workload(w)
        recs = [g.trial() for _ in range(40)]
    o = O.OracleSystem.from_workload(w, cap=w.n + 64)
    n_inst = n_acc = 0
    for t, rg in enumerate(recs):
        ro = o.trial(t)
        assert rg["move"] == ro["move"] and rg["n_steps"] == ro["n_steps"], (t, rg, ro)
        assert rg["flags"] & 0x13 == ro["flags"], (t, rg["flags"], ro["flags"])
        if not ro["flags"] & 0x3:
            for key in ("dH", "W_prot", "E_switch", "H0", "H1"):
                assert abs(rg[key] - ro[key]) <= 1e-6 * max(1.0, abs(ro[key])), (t, key, rg[key], ro[key])
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        n_inst += bool(ro["flags"] & O.FLAG_INSTANT)
        n_acc += ro["accepted"]
    say(f"   instant {n_inst}, accepted {n_acc} of 40")
    assert n_inst > 0 and n_acc > 0
    g.close()


def test_early_rejection_excludes_the_learned_proposal():
    w = W.lj_electrolyte(300, 0.1, 79, n_steps=20, precision="fp64")
    w.params.update(v_ex_edge=7.0)
    g = h4d.System.from_workload(w)
    with pytest.raises(h4d.H4DError) as e:
        g.set_proposal(None, 4)
    assert e.value.code == h4d.H4D_EINVAL
    g.close()
