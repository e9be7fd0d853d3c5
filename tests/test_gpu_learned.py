"""GPU parity of the learned proposal: site features (FP32, fixed-point
sums) against the FP64 oracle, BF16 matrix-core inference and FP32
forward, backpropagation and Adam against the FP64 network, trial
decisions replayed through the oracle, the ideal-gas laws under a biased
proposal, and the gain of a trained network over the uniform proposal.

Tolerances:
* features: |f_gpu - f_ref| <= 2e-4 (1 + |f_ref|) (FP32 terms, continuous features);
* FP32 logits: 1e-4 relative to the spread of the reference logits;
  BF16 logits: 3e-2 of it (8-bit mantissas through three layers);
* gradients: ||g_gpu - g_ref|| <= 1e-4 ||g_ref||;
* replayed trials (FP64 trajectories, the GPU's logits fed to the oracle):
  identical moves, sites and decisions; ln_proposal within 1e-12, dH within
  1e-6 relative.
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


def random_sites(rng, n, L):
    return rng.uniform(0.0, L, size=(n, 6))


@pytest.mark.parametrize("kind", ["lj", "water"])
def test_site_features_match_oracle(kind):
    say(f"case site features {kind}")
    if kind == "lj":
        w = W.lj_electrolyte(1500, 0.3, 61, precision="fp32")
        w.params.update(kappa_sr=0.6)
    else:
        w = W.water_nacl(n_water=300, n_pairs=10, L=21.0, m=7, seed=62)
        w.params.update(precision="fp32")
    L = w.params["box"][0]
    rng = np.random.default_rng(7)
    sites = random_sites(rng, 200, L)
    g = h4d.System.from_workload(w)
    fg = g.site_features(sites)
    o = O.OracleSystem.from_workload(w)
    fr = np.array([o.site_features(s) for s in sites])
    err = np.abs(fg - fr) / (1.0 + np.abs(fr))
    say(f"   worst scaled feature difference {err.max():.3e} (feature {np.unravel_index(err.argmax(), err.shape)[1]})")
    assert err.max() <= 2e-4
    g.close()


def test_mlp_inference_and_fp32_forward_match_fp64():
    say("case network forward: BF16 matrix cores and FP32 vs FP64 (333 rows)")
    rng = np.random.default_rng(11)
    theta = mlp.random_theta(21, scale=1.3)
    theta[mlp.N_PARAMS - 129:mlp.N_PARAMS - 1] *= 2.0
    X = rng.normal(size=(333, 64)) * np.linspace(0.3, 3.0, 64)
    ref = mlp.forward(theta, X)
    net = h4d.Mlp(seed=1)
    net.set_weights(theta)
    s32 = net.forward(X, bf16=False)
    s16 = net.forward(X, bf16=True)
    spread = max(1.0, float(np.std(ref)))
    e32 = np.abs(s32 - ref).max() / spread
    e16 = np.abs(s16 - ref).max() / spread
    say(f"   logit spread {spread:.3f}; FP32 worst {e32:.2e}; BF16 worst {e16:.2e}")
    assert e32 <= 1e-4
    assert e16 <= 3e-2
    # the weights read back are the weights set (FP32 round trip)
    assert np.array_equal(net.weights(), theta.astype(np.float32))
    net.close()


def test_mlp_gradient_and_adam_match_fp64():
    say("case network backpropagation and Adam vs FP64 (200 rows)")
    rng = np.random.default_rng(12)
    theta = mlp.random_theta(22, scale=1.0)
    X = rng.normal(size=(200, 64))
    t = rng.normal(size=200) * 3.0
    net = h4d.Mlp(seed=2)
    net.set_weights(theta)
    lg, gg = net.loss_grad(X, t)
    th32 = theta.astype(np.float32).astype(np.float64)
    lr_, gr = mlp.loss_and_grad(th32, X.astype(np.float32).astype(np.float64), t.astype(np.float32))
    rel = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
    say(f"   loss {lg:.6f} vs {lr_:.6f}; gradient relative difference {rel:.2e}")
    assert lg == pytest.approx(lr_, rel=1e-5)
    assert rel <= 1e-4
    # five full-batch Adam steps, in standardized input coordinates (the
    # documented procedure of the training call), mapped back to raw features
    net.train(X, t, steps=5, batch=200, lr=1e-3, seed=3)
    X32 = X.astype(np.float32).astype(np.float64)
    mean, sd = mlp.standardization(X32)
    Xs = (X32 - mean) / sd
    th = mlp.to_standard(th32, mean, sd)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in range(1, 6):
        _, g = mlp.loss_and_grad(th, Xs, t.astype(np.float32))
        th, m, v = mlp.adam_step(th, m, v, g, step, 1e-3)
    th = mlp.from_standard(th, mean, sd)
    d_gpu = net.weights().astype(np.float64) - th32
    d_ref = th - th32
    rel = np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref)
    say(f"   Adam update relative difference {rel:.2e}")
    assert rel <= 1e-2
    net.close()


@pytest.mark.parametrize("scale", [1.0, 0.5])
def test_learned_trials_replay_oracle_decisions(scale):
    say(f"case learned trials fp64 lj500, k = 32, weight scale {scale}, replayed through the oracle")
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0, n_steps=60)
    k = 32
    theta = mlp.random_theta(31, scale=2.0)
    net = h4d.Mlp(seed=3)
    net.set_weights(theta)
    g = h4d.System.from_workload(w)
    g.set_proposal(net, k, 10.0, scale)
    o = O.OracleSystem.from_workload(w, cap=w.n + 200)
    worst_feat = 0.0
    n_acc = 0
    for t in range(14):
        rg = g.trial()
        sites, fg, lg = g.last_candidates(k)
        seen = {}

        def replay(X):
            seen["X"] = X
            return lg.astype(np.float64)

        ro, _ = o.trial_learned(t, k, replay, scale=scale)
        assert rg["move"] == ro["move"] and rg["flags"] & 3 == ro["flags"]
        if ro["flags"] & 1:
            continue
        assert "X" in seen
        err = np.abs(fg - seen["X"]) / (1.0 + np.abs(seen["X"]))
        worst_feat = max(worst_feat, float(err.max()))
        assert rg["ln_proposal"] == pytest.approx(ro["ln_proposal"], rel=1e-12, abs=1e-12)
        for key in ("dH", "W_prot", "E_switch", "H0"):
            assert abs(rg[key] - ro[key]) <= 1e-6 * max(1.0, abs(ro[key])), (t, key)
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        n_acc += rg["accepted"]
    say(f"   accepted {n_acc} of 14; worst candidate feature difference {worst_feat:.2e}")
    assert worst_feat <= 2e-4
    st = g.state()
    assert st["n"] == o.n and np.array_equal(st["tag"], o.tag[: o.n])
    g.close()
    net.close()


def crafted_bias_theta():
    """A network whose logit grows as the sites near existing ions: hidden
    unit 0 carries 10 - 4 d_c - 4 d_a + 2 r_ca (distances over rc) through
    the three GELU layers; every other unit is zero."""
    th = np.zeros(mlp.N_PARAMS)
    H = 128
    oW1, ob1 = 0, 64 * H
    oW2 = ob1 + H
    oW3 = oW2 + H * H + H
    ow4 = oW3 + H * H + H
    th[oW1 + 29 * H + 0] = -4.0
    th[oW1 + 60 * H + 0] = -4.0
    th[oW1 + 62 * H + 0] = 2.0
    th[ob1 + 0] = 10.0
    th[oW2 + 0] = 1.0
    th[oW3 + 0] = 1.0
    th[ow4 + 0] = 1.0
    th[-1] = -8.0
    return th


def test_ideal_gas_laws_under_a_biased_learned_proposal():
    say("case ideal gas, biased learned proposal k = 8 (20000 trials)")
    y, L, r0 = 3.0, 5.0, 1.5
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    w.params.update(capacity=256)
    net = h4d.Mlp(seed=4)
    net.set_weights(crafted_bias_theta())
    g = h4d.System.from_workload(w)
    g.set_proposal(net, 8)
    ns, lnq = [], []
    close = pairs = 0
    for chunk in range(40):
        recs = g.trials(500, as_array=True)
        for q in range(500):
            ns.append(recs[q].n_salt_after)
            if recs[q].move > 0:
                lnq.append(recs[q].ln_proposal)
        if chunk >= 2:
            st = g.state()
            x = st["x"]
            if len(x) >= 2:
                d = x[:, None, :] - x[None, :, :]
                d -= L * np.round(d / L)
                dist = np.linalg.norm(d, axis=2)[np.triu_indices(len(x), 1)]
                close += int((dist < r0).sum())
                pairs += len(dist)
    # positions are sampled once per 500 trials; add more samples in short runs
    for q in range(1500):
        g.trials(4)
        x = g.state()["x"]
        if len(x) >= 2:
            d = x[:, None, :] - x[None, :, :]
            d -= L * np.round(d / L)
            dist = np.linalg.norm(d, axis=2)[np.triu_indices(len(x), 1)]
            close += int((dist < r0).sum())
            pairs += len(dist)
    ns = np.array(ns[1000:])
    n = np.arange(60)
    logp = 2 * n * math.log(y) - 2 * np.array([math.lgamma(k + 1) for k in n])
    exact = np.exp(logp - logp.max())
    exact /= exact.sum()
    emp = np.bincount(ns, minlength=60)[:60] / len(ns)
    tv = 0.5 * np.abs(emp - exact).sum()
    p_close = 4.0 / 3.0 * math.pi * r0 ** 3 / L ** 3
    say(f"   TV {tv:.4f}; close-pair fraction {close / pairs:.4f} (uniform {p_close:.4f}); "
        f"std ln q {np.std(lnq):.2f}")
    assert tv < 0.03
    assert abs(close / pairs - p_close) < 0.1 * p_close
    assert np.std(lnq) > 0.5
    g.close()
    net.close()


def test_trained_network_raises_insertion_acceptance():
    """A state where insertion sites really differ: 2,000 LJ ions at density
    0.45 fill half of an elongated box (a dense slab beside empty space).
    Pilot insertions with the uniform proposal (k = 1, equal weights, never
    accepted: the state stays fixed) record each site's features and dH; the
    network learns clip(-beta dH, -20, 10) on the GPU; from the same state,
    learned insertions (k = 16) are compared with uniform ones.  The share of
    insertions with a prohibitive work (beta dH > 20, a site inside the
    slab) must fall by half.  Under any proposal the multiple-try ratio has
    the uniform ratio's mean, so the mean acceptance probability can only
    rise where uniform ratios exceed 1 and are cut off by min(1, R): that is
    asserted 8 units of beta mu above the operating point (the beta mu at
    which the pilot's mean insertion ratio is 1); the whole scan is printed."""
    say("case learned vs uniform insertions, slab of 2000 LJ ions beside empty space, fp32, N_f = 100")
    w = W.lj_electrolyte(2000, 0.45, 81, n_steps=100, precision="fp32")
    a = w.params["box"][0]
    w.params.update(box=[2.0 * a, a, a], beta_mu=-1000.0)
    g = h4d.System.from_workload(w)
    g.set_proposal(None, 1)
    feats, dH = [], []
    for t in range(1000):
        r = g.trial(h4d.MOVE_INSERT)
        assert not r["accepted"]
        feats.append(g.last_site_features())
        dH.append(r["dH"])
    X = np.array(feats)
    dH = np.array(dH)
    beta = 1.0 / w.params["kT"]
    y = np.clip(-beta * dH, -20.0, 10.0)
    net = h4d.Mlp(seed=5)
    losses = net.train(X, y, steps=2000, batch=256, lr=1e-3, seed=6)
    say(f"   training loss {losses[:10].mean():.2f} -> {losses[-50:].mean():.2f}; target spread {y.std():.2f}")
    assert losses[-50:].mean() < 0.3 * losses[:10].mean()
    V = 2.0 * a ** 3
    I = 2.0 * math.log(V / (w.nsalt + 1))
    m = (-beta * dH).max()
    bmu = -I - (m + math.log(np.mean(np.exp(-beta * dH - m))))

    def mean_acc(records, beta_mu):
        lnR = np.array([r["ln_ratio"] for r in records]) + 1000.0 + beta_mu
        return float(np.mean(np.exp(np.minimum(lnR, 0.0))))

    g.set_trial_index(100000)
    g.set_proposal(None, 0)
    plain = [g.trial(h4d.MOVE_INSERT) for _ in range(500)]
    g.set_trial_index(200000)
    g.set_proposal(net, 16)
    learned = [g.trial(h4d.MOVE_INSERT) for _ in range(500)]
    bad_p = np.mean([beta * r["dH"] > 20.0 for r in plain])
    bad_l = np.mean([beta * r["dH"] > 20.0 for r in learned])
    say(f"   insertions with beta dH > 20: uniform {bad_p:.3f}, learned {bad_l:.3f}")
    gains = {}
    for bm in (bmu - 2.0, bmu, bmu + 2.0, bmu + 4.0, bmu + 6.0, bmu + 8.0):
        a_p, a_l = mean_acc(plain, bm), mean_acc(learned, bm)
        gains[bm] = a_l / max(a_p, 1e-12)
        say(f"   beta mu {bm:.2f}: mean insertion acceptance uniform {a_p:.4f}, learned {a_l:.4f} "
            f"(x{gains[bm]:.2f})")
    assert bad_l < 0.5 * bad_p
    assert gains[bmu + 8.0] > 1.3
    g.close()
    net.close()
