"""Pins of the oracle's learned proposal: the site features, the
multiple-try acceptance factor and the FP64 network.

The features are this project's definition (any deterministic function of
the state keeps the method exact).  They are pinned to facts that hold by
construction, not to a second copy of their formulas:
* invariance under translation of everything and under permutation of the atoms;
* a lone atom in a large box gives one exact Gaussian shell value;
* the energy features add up to the energy of the ion flying at w = 0 and
  at w = w_max, computed by the independent pair sum (mode FLY);
* the Coulomb force feature is the gradient of the Coulomb energy feature
  (central differences);
* the pair features come from the two-ion system's energy.
The multiple-try factor is pinned by the ideal-gas laws (of N, and of the
uniform placement of the ions) under a strongly biased proposal, and by its
reduction to the uniform proposal.  The
network is pinned by finite differences, the exact (erf) GELU, closed forms
at zero weights, Adam's first step, and the invariance of its function
under the change to standardized input coordinates.
"""
import math

import numpy as np
import pytest
from scipy.special import i0, i1

from oracle import mlp
from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def lj_state(n=300, rho=0.3, seed=41, **kw):
    w = W.lj_electrolyte(n, rho, seed, precision="fp64")
    w.params.update(kappa_sr=0.7, **kw)
    return w


def unscaled(f):
    return np.sinh(f)


def test_features_translation_and_permutation_invariant():
    w = lj_state()
    L = w.params["box"][0]
    site = np.array([1.3, 7.2, 3.3, 5.5, 0.4, 9.9])
    f0 = O.OracleSystem.from_workload(w).site_features(site)
    shift = np.array([2.1, -3.7, 5.05])
    w2 = lj_state()
    w2.x = np.mod(w.x + shift, L)
    f1 = O.OracleSystem.from_workload(w2).site_features(np.mod(site + np.tile(shift, 2), L))
    assert np.allclose(f0, f1, rtol=1e-10, atol=1e-10)
    perm = np.random.default_rng(0).permutation(w.n)
    w3 = lj_state()
    w3.x, w3.type = w.x[perm], w.type[perm]
    f2 = O.OracleSystem.from_workload(w3).site_features(site)
    assert np.allclose(f0, f2, rtol=1e-12, atol=1e-12)


def test_lone_atom_gives_one_gaussian_shell():
    # one anion at distance (m + 1/2) rc / 6 from the cation site: that shell
    # holds exactly the taper (1 - r^2/rc^2)^2, its neighbours exp(-2) times
    # it, the next exp(-8) times it
    w = W.small_lj(2, 0.3, 3)
    L = 40.0
    p = dict(w.params, box=[L, L, L])
    rc = max(p["rc_lj"], p["rc_coul"])
    m = 3
    r = (m + 0.5) * rc / 6
    x = np.array([[10.0 + r, 10.0, 10.0]])
    s = O.OracleSystem(p, x, np.array([1], np.int32), np.array([-1], np.int32), np.array([0], np.int64), 0)
    f = s.site_features([10.0, 10.0, 10.0, 30.0, 30.0, 30.0])
    shells = f[:24].reshape(4, 6)
    taper = (1.0 - (r / rc) ** 2) ** 2
    assert shells[1, m] == pytest.approx(0.1 * taper, rel=1e-14)
    assert shells[1, m - 1] == pytest.approx(0.1 * taper * math.exp(-2.0), rel=1e-12)
    assert shells[1, m + 1] == pytest.approx(0.1 * taper * math.exp(-2.0), rel=1e-12)
    assert shells[1, m - 2] == pytest.approx(0.1 * taper * math.exp(-8.0), rel=1e-12)
    assert np.all(shells[0] == 0.0) and np.all(shells[2:] == 0.0)
    assert f[29] == pytest.approx(r / rc, rel=1e-14)      # nearest atom
    assert f[30] == pytest.approx(r / rc, rel=1e-14)      # nearest counter-ion (an anion)
    assert f[31 + 29] == 1.0                               # the anion site sees nobody within rc


@pytest.mark.parametrize("which", [0, 1])
def test_energy_features_equal_the_flying_ion_energy(which):
    w = lj_state()
    p = w.params
    beta = 1.0 / p["kT"]
    site = np.array([3.1, 4.4, 8.8, 6.0, 2.2, 1.7])
    f = O.OracleSystem.from_workload(w).site_features(site)
    g = f[31 * which:31 * which + 31]
    # the same ion appended as the only flying atom: pair sum of mode FLY
    ion_type = p["cation_type"] if which == 0 else p["anion_type"]
    x = np.vstack([w.x, site[3 * which:3 * which + 3]])
    t = np.append(w.type, ion_type).astype(np.int32)
    s = O.OracleSystem(p, x, t, np.full(len(t), -1, np.int32), np.arange(len(t), dtype=np.int64), w.nsalt)
    s.flying[len(t) - 1] = 1
    e0, _ = s.compute(0.0, O.MODE_FLY, forces=False)
    ew, _ = s.compute(p["w_max"], O.MODE_FLY, forces=False)
    assert unscaled(g[24]) + unscaled(g[26]) == pytest.approx(beta * e0.U, rel=1e-9, abs=1e-9)
    assert unscaled(g[27]) + unscaled(g[28]) == pytest.approx(beta * ew.U, rel=1e-9, abs=1e-9)
    assert unscaled(g[26]) == pytest.approx(beta * e0.U_lj, rel=1e-9, abs=1e-9)


def test_coulomb_force_feature_is_gradient_of_coulomb_energy():
    w = lj_state()
    o = O.OracleSystem.from_workload(w)
    site = np.array([2.7, 5.9, 6.3, 8.1, 1.1, 4.0])
    f = o.site_features(site)
    h = 1e-6
    grad = np.zeros(3)
    for c in range(3):
        sp, sm = site.copy(), site.copy()
        sp[c] += h
        sm[c] -= h
        grad[c] = (unscaled(o.site_features(sp)[24]) - unscaled(o.site_features(sm)[24])) / (2 * h)
    assert unscaled(f[25]) == pytest.approx(np.linalg.norm(grad), rel=1e-6)


def test_pair_features_from_the_two_ion_system():
    w = W.small_lj(2, 0.3, 3)
    L = 30.0
    p = dict(w.params, box=[L, L, L])
    rc = max(p["rc_lj"], p["rc_coul"])
    site = np.array([5.0, 5.0, 5.0, 6.2, 5.9, 4.6])
    r = np.linalg.norm(site[3:] - site[:3])
    empty = O.OracleSystem(p, np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros(0, np.int32),
                           np.zeros(0, np.int64), 0)
    f = empty.site_features(site)
    two = O.OracleSystem(p, site.reshape(2, 3), np.array([0, 1], np.int32), np.array([-1, -1], np.int32),
                         np.array([0, 1], np.int64), 1)
    e, _ = two.compute(0.0, forces=False)
    assert f[62] == pytest.approx(r / rc, rel=1e-14)
    assert unscaled(f[63]) == pytest.approx(e.U / p["kT"], rel=1e-10)
    # an empty box: no shell counts, no energies, nearest distances capped
    assert np.all(f[:24] == 0.0) and np.all(f[24:29] == 0.0) and f[29] == 1.0 and f[30] == 1.0


def test_equal_weights_and_single_candidate_reduce_to_the_uniform_proposal():
    w = lj_state(n=200, rho=0.25, n_steps=20)
    theta = mlp.random_theta(5, scale=3.0)
    a = O.OracleSystem.from_workload(w, cap=w.n + 40)
    b = O.OracleSystem.from_workload(w, cap=w.n + 40)
    for t in range(6):
        ra, _ = a.trial_learned(t, 8, None)
        rb, _ = b.trial_learned(t, 1, lambda X: mlp.forward(theta, X))
        assert ra["ln_proposal"] == 0.0 and rb["ln_proposal"] == 0.0


def test_zero_weight_scale_is_the_equal_weight_proposal():
    # log weights scale * min(s, cap): scale 0 makes every candidate's weight
    # 1 whatever the network says, so the trials repeat the equal-weight run
    # record for record; a positive scale moves ln q away from 0
    w = lj_state(n=200, rho=0.25, n_steps=20)
    theta = mlp.random_theta(5, scale=3.0)
    net = lambda X: mlp.forward(theta, X)
    a = O.OracleSystem.from_workload(w, cap=w.n + 40)
    b = O.OracleSystem.from_workload(w, cap=w.n + 40)
    c = O.OracleSystem.from_workload(w, cap=w.n + 40)
    lnq = []
    for t in range(6):
        ra, fa = a.trial_learned(t, 8, None)
        rb, fb = b.trial_learned(t, 8, net, scale=0.0)
        assert ra == rb and np.array_equal(fa, fb)
        rc, _ = c.trial_learned(t, 8, net, scale=0.5)
        lnq.append(rc["ln_proposal"])
    assert np.array_equal(a.positions(), b.positions())
    assert max(abs(q) for q in lnq) > 1e-3


def test_ideal_gas_laws_hold_under_a_biased_proposal():
    # a proposal that strongly prefers sites next to existing ions (any
    # weights keep the chain exact): N still follows y^(2N) / (N!)^2 and the
    # ions stay uniformly and independently placed, so the fraction of ion
    # pairs closer than r0 is (4/3) pi r0^3 / V.  Without the multiple-try
    # factor the positions cluster (that fraction grows by more than half).
    y, L, r0 = 3.0, 5.0, 1.5
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    s = O.OracleSystem.from_workload(w, cap=256, use_cells=False)

    def bias(X):
        return 4.0 * (2.0 - X[:, 29] - X[:, 31 + 29]) + 2.0 * X[:, 62]

    ns, lnq = [], []
    close = pairs = 0
    for t in range(30000):
        r, _ = s.trial_learned(t, 8, bias)
        ns.append(s.nsalt)
        if r["move"] > 0:
            lnq.append(r["ln_proposal"])
        if t >= 1000 and t % 4 == 0 and s.n >= 2:
            x = s.positions()
            d = x[:, None, :] - x[None, :, :]
            d -= L * np.round(d / L)
            dist = np.linalg.norm(d, axis=2)[np.triu_indices(s.n, 1)]
            close += int((dist < r0).sum())
            pairs += len(dist)
    ns = np.array(ns[1000:])
    n = np.arange(60)
    logp = 2 * n * math.log(y) - 2 * np.array([math.lgamma(k + 1) for k in n])
    exact = np.exp(logp - logp.max())
    exact /= exact.sum()
    emp = np.bincount(ns, minlength=60)[:60] / len(ns)
    assert 0.5 * np.abs(emp - exact).sum() < 0.02
    assert ns.mean() == pytest.approx(y * i1(2 * y) / i0(2 * y), abs=0.06)
    p_close = 4.0 / 3.0 * math.pi * r0 ** 3 / L ** 3
    assert abs(close / pairs - p_close) < 0.1 * p_close
    assert np.std(lnq) > 0.5          # the proposal is far from uniform


def test_gelu_is_close_to_the_exact_gelu():
    x = np.linspace(-5, 5, 2001)
    exact = 0.5 * x * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in x]))
    assert np.abs(mlp.gelu(x) - exact).max() < 1e-3
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = mlp.random_theta(7, scale=1.5)
    X = rng.normal(size=(5, 64))
    t = rng.normal(size=5)
    loss, g = mlp.loss_and_grad(theta, X, t)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1, 64 * 128 + 3]])
    h = 1e-6
    for q in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[q] += h
        tm[q] -= h
        fd = (mlp.loss_and_grad(tp, X, t)[0] - mlp.loss_and_grad(tm, X, t)[0]) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_zero_network_closed_forms_and_first_adam_step():
    theta = np.zeros(mlp.N_PARAMS)
    c = 0.7
    theta[-1] = c                           # output bias
    X = np.random.default_rng(1).normal(size=(9, 64))
    t = np.linspace(-2, 3, 9)
    loss, g = mlp.loss_and_grad(theta, X, t)
    assert loss == pytest.approx(np.mean((c - t) ** 2), rel=1e-14)
    assert g[-1] == pytest.approx(2 * np.mean(c - t), rel=1e-14)
    assert np.all(g[:-1 - 128] == 0.0)      # everything behind a zero output layer
    th1, m, v = mlp.adam_step(theta, np.zeros_like(g), np.zeros_like(g), g, 1, 1e-3)
    # first bias-corrected step: -lr * g / (|g| + eps)
    assert th1[-1] - theta[-1] == pytest.approx(-1e-3 * np.sign(g[-1]), rel=1e-6)
    assert mlp.N_PARAMS == 41473


def test_standardized_coordinates_leave_the_network_unchanged():
    rng = np.random.default_rng(9)
    theta = mlp.random_theta(11)
    X = rng.normal(size=(40, 64)) * rng.uniform(0.1, 30.0, size=64) + rng.normal(size=64) * 5
    mean, sd = mlp.standardization(X)
    ts = mlp.to_standard(theta, mean, sd)
    assert np.allclose(mlp.forward(ts, (X - mean) / sd), mlp.forward(theta, X), rtol=1e-10, atol=1e-10)
    assert np.allclose(mlp.from_standard(ts, mean, sd), theta, rtol=1e-12, atol=1e-12)
