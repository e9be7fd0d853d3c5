"""GPU parity of the bimodal bias of the flying pair's separation (Sec.
II B 4, Eqs. 12-16): biased insertion offsets, B_ins-weighted deletion
choice and the B_del / B_ins factors follow the oracle trial by trial, and
the biased chain on the GPU keeps the ideal-gas laws."""
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


def test_biased_fp64_trials_match_oracle_sequence():
    say("case trials lj500 fp64 with the bimodal bias (x_b 1.2, alpha_b 2), 30 trials")
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0, bias_xb=1.2, bias_alpha=2.0)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 200)
    n_acc = 0
    for t in range(30):
        rg, ro = g.trial(), o.trial(t)
        assert rg["move"] == ro["move"] and rg["flags"] & 3 == ro["flags"]
        assert rg["tag_c"] == ro["tag_c"] and rg["tag_a"] == ro["tag_a"], (t, rg, ro)
        if not ro["flags"]:
            assert rg["ln_proposal"] == pytest.approx(ro["ln_proposal"], rel=1e-10, abs=1e-10), t
            for key in ("dH", "W_prot", "E_switch", "H0"):
                assert abs(rg[key] - ro[key]) <= 1e-6 * max(1.0, abs(ro[key])), (t, key)
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        n_acc += rg["accepted"]
    say(f"   accepted {n_acc} of 30")
    st = g.state()
    assert st["n"] == o.n and np.array_equal(st["tag"], o.tag[: o.n])
    d = st["x"] - o.x[: o.n]
    L = w.params["box"][0]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-8
    g.close()


def test_bias_switches_and_limits():
    w = W.config_lj_500()
    g = h4d.System.from_workload(w)
    with pytest.raises(h4d.H4DError):
        g.set_bias(5.0, 2.0)            # reach beyond half an edge (L = 11.9)
    with pytest.raises(h4d.H4DError):
        g.set_bias(1.0, -1.0)
    g.set_bias(1.2, 2.0)
    r = g.trial(h4d.MOVE_INSERT)
    assert r["ln_proposal"] != 0.0
    g.set_bias(0.0, 0.0)
    r = g.trial(h4d.MOVE_INSERT)
    assert r["ln_proposal"] == 0.0
    g.close()


def test_ideal_gas_laws_under_the_bias_on_gpu():
    say("case ideal gas with the bimodal bias (x_b 0.5, alpha_b 6), 40,000 trials")
    y, L, r0 = 3.0, 5.0, 1.0
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    w.params.update(capacity=256, bias_xb=0.5, bias_alpha=6.0)
    g = h4d.System.from_workload(w)
    cat, an = w.params["cation_type"], w.params["anion_type"]
    ns, lnq = [], []
    close = pairs = 0
    for chunk in range(80):
        recs = g.trials(500, as_array=True)
        for q in range(500):
            ns.append(recs[q].n_salt_after)
            lnq.append(recs[q].ln_proposal)
        if chunk >= 2:
            for _ in range(20):
                g.trials(3)
                st = g.state()
                xc, xa = st["x"][st["type"] == cat], st["x"][st["type"] == an]
                if len(xc) and len(xa):
                    d = xc[:, None, :] - xa[None, :, :]
                    d -= L * np.round(d / L)
                    dist = np.linalg.norm(d, axis=2).ravel()
                    close += int((dist < r0).sum())
                    pairs += dist.size
    ns = np.array(ns[1000:])
    n = np.arange(60)
    logp = 2 * n * math.log(y) - 2 * np.array([math.lgamma(k + 1) for k in n])
    exact = np.exp(logp - logp.max())
    exact /= exact.sum()
    emp = np.bincount(ns, minlength=60)[:60] / len(ns)
    tv = 0.5 * np.abs(emp - exact).sum()
    p_close = 4.0 / 3.0 * math.pi * r0 ** 3 / L ** 3
    say(f"   TV {tv:.4f}; cation-anion close fraction {close / pairs:.4f} (uniform {p_close:.4f}); "
        f"std ln q {np.std(lnq):.2f}")
    assert tv < 0.03
    assert abs(close / pairs - p_close) < 0.1 * p_close
    assert np.std(lnq) > 0.5
    g.close()
