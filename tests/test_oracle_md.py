"""Pins of the oracle's equilibrium phase between trials (generalized hybrid
MC) and of the trials that carry the state's momenta with the symmetric
two-end momentum reversal (Sec. II A).

- the phase's velocity Verlet conserves H to second order in dt;
- a rejected phase keeps the positions and reverses the refreshed momenta;
- a pair of neutral LJ atoms sampled by the phase alone follows the
  canonical pair density r^2 exp(-beta U(r)) (quadrature of the oracle's
  pair potential), with kinetic temperature kT, for a full and a partial
  momentum refresh;
- a rejected trial with carried momenta leaves the positions and each
  momentum times one common sign, -1 in about half of the trials;
- with carried momenta the ideal reservoir keeps its closed-form
  distribution of N, and an interacting electrolyte reaches the same mean N
  as with fresh momenta (both samplers are exact)."""
import math

import numpy as np
import pytest
from scipy.special import i0, i1

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def _phase_dH(dt, T_total=0.4):
    # like charges without LJ (a force continuous at the cutoff): velocity
    # Verlet's energy error is O(dt^2)
    w = W.lj_electrolyte(200, 0.3, 9)
    w.params.update(dt=dt, charge=[1.0, 1.0], eps=[0.0, 0.0], md_refresh=0.0)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    r = s.md_phase(3, int(round(T_total / dt)))
    return abs(r["dH"])


def test_phase_energy_error_is_second_order():
    d1, d2 = _phase_dH(0.004), _phase_dH(0.002)
    assert 2.5 < d1 / d2 < 6.0


def test_phase_metropolis_and_rejection_bookkeeping():
    # a large step makes rejections common
    w = W.lj_electrolyte(200, 0.3, 4)
    w.params.update(dt=0.02, md_refresh=0.3)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    seen = {0: 0, 1: 0}
    for t in range(40):
        x0, v0 = s.positions(), s.velocities()
        r = s.md_phase(t, 10)
        assert r["move"] == 2 and r["trial"] == t and r["n_steps"] == 10
        assert r["accepted"] == int(r["ln_u"] < -r["dH"] / w.params["kT"])
        assert r["ln_ratio"] == pytest.approx(-r["dH"] / w.params["kT"])
        seen[r["accepted"]] += 1
        if not r["accepted"]:
            assert np.array_equal(s.positions(), x0)
            # the refreshed momenta, reversed: v = -(c v0 + sqrt(1 - c^2) xi)
            c = 0.3
            xi = (-s.velocities() - c * v0) / math.sqrt(1 - c * c)
            assert abs(np.mean(xi * xi) - 1.0) < 0.35     # a unit normal draw (m = kT = 1)
        else:
            assert not np.array_equal(s.positions(), x0)
    assert seen[0] > 3 and seen[1] > 3


def _pair_density_probability(params, r_split, r_max):
    r = np.linspace(1e-3, r_max, 40001)
    u = np.array([sum(O.pair(params, 0, 0, x)[:2]) for x in r])
    f = r * r * np.exp(-u / params["kT"])
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(r))])
    return np.interp(r_split, r, cum) / cum[-1]


@pytest.mark.parametrize("refresh", [0.0, 0.6])
def test_phase_samples_the_canonical_pair_density(refresh):
    L = 5.2
    p = W._base_lj_params(L)
    p.update(charge=[0.0, 0.0], rc_coul=2.5, dt=0.01, md_refresh=refresh, seed=21)
    x = np.array([[1.0, 1.0, 1.0], [2.3, 1.0, 1.0]])
    s = O.OracleSystem(p, x, np.array([0, 0], np.int32), np.array([-1, -1], np.int32),
                       np.array([0, 1], np.int64), 0, use_cells=False)
    r_all, v2 = [], []
    for t in range(20000):
        s.md_phase(t, 40)
        d = s.x[1] - s.x[0]
        d -= L * np.round(d / L)
        r_all.append(np.sqrt(d @ d))
        v2.append(np.mean(s.velocities() ** 2))
    r_all = np.array(r_all[200:])
    inside = r_all[r_all < 0.5 * L]
    emp = np.mean(inside < 1.5)
    exact = _pair_density_probability(p, 1.5, 0.5 * L)
    assert emp == pytest.approx(exact, abs=0.025)
    assert np.mean(v2) == pytest.approx(1.0, abs=0.04)      # m <v^2> = kT per component


def test_rejected_trial_with_carried_momenta_reverses_them_by_one_sign():
    w = W.lj_electrolyte(60, 0.1, 6, n_steps=10)
    w.params.update(beta_mu=-40.0, momenta=1)        # insertions all but never accepted
    s = O.OracleSystem.from_workload(w, use_cells=False)
    signs = []
    for t in range(200):
        x0, v0 = s.positions(), s.velocities()
        r = s.trial(t, +1)
        assert not r["accepted"]
        assert np.array_equal(s.positions(), x0)
        v1 = s.velocities()
        sg = 1.0 if np.array_equal(v1, v0) else -1.0
        assert np.array_equal(v1, sg * v0)
        signs.append(sg)
    n_neg = signs.count(-1.0)
    assert 70 < n_neg < 130                           # Binomial(200, 1/2)


def test_accepted_insertion_keeps_the_trajectory_momenta():
    # kinetic energy of the old atoms after an accepted insertion with carried
    # momenta: K_start + dK, K_start that of the carried momenta
    w = W.lj_electrolyte(60, 0.1, 6, n_steps=10)
    w.params.update(beta_mu=60.0, momenta=1)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    n0 = s.n
    K0 = 0.5 * np.sum(s.velocities() ** 2)
    r = s.trial(0, +1)
    assert r["accepted"]
    K_old = 0.5 * np.sum(s.velocities()[:n0] ** 2)
    assert K_old == pytest.approx(K0 + r["dK"], rel=1e-12)


def test_ideal_reservoir_with_carried_momenta_and_phases():
    y, L = 3.0, 5.0
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    w.params.update(momenta=1, md_refresh=0.5)
    s = O.OracleSystem.from_workload(w, cap=256, use_cells=False)
    ns = []
    for t in range(40000):
        if t % 4 == 0 and s.n:
            assert s.md_phase(t, 2)["accepted"]       # free flight: dH = 0
        s.trial(t)
        ns.append(s.nsalt)
    ns = np.array(ns[1000:])
    assert ns.mean() == pytest.approx(y * i1(2 * y) / i0(2 * y), abs=0.08)


def _gc_mean_n(momenta, n, seed=5):
    w = W.lj_electrolyte(20, 0.02, seed, n_steps=10)
    w.params.update(beta_mu=-10.5, momenta=momenta, md_refresh=0.5, dt=0.01)
    s = O.OracleSystem.from_workload(w, cap=400, use_cells=False)
    N = []
    for t in range(n):
        s.md_phase(t, 5)
        s.trial(t)
        N.append(s.nsalt)
    N = np.array(N[1000:], dtype=float)
    nb = 25
    b = N[: len(N) // nb * nb].reshape(nb, -1).mean(1)
    return N.mean(), b.std(ddof=1) / math.sqrt(nb)


def test_carried_and_fresh_momenta_sample_the_same_reservoir():
    m0, e0 = _gc_mean_n(0, 16000)
    m1, e1 = _gc_mean_n(1, 16000)
    assert abs(m0 - m1) < 4.0 * math.hypot(e0, e1) + 0.05
