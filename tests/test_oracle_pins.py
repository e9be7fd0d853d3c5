"""Pins of the FP64 CPU oracle against facts that do not come from the
oracle itself: a published generator, closed forms of the potentials,
calculus (finite differences), conservation laws, time reversibility and
the exact stationary distribution of an ideal ion-pair reservoir."""
import json
import ctypes
import math
import os

import numpy as np
import pytest
from scipy.special import erfc, i0, i1

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Counter-based generator: numpy ships an independent Philox4x64-10.
# numpy increments the 256-bit counter before each block, so its first
# block for counter c equals the published function at c + 1.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 2, 77, 0), (1001, 3)),
    ((123456789, 1, 2**40 + 7, 9), (2**63 + 5, 17)),
    ((2**64 - 1, 0, 0, 0), (1, 2)),
])
def test_philox_matches_numpy(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    # step numpy's counter back by one (with borrow) so its next block is ctr
    prev = [int(v) for v in c]
    i = 0
    while True:
        if prev[i] > 0:
            prev[i] -= 1
            break
        prev[i] = 2**64 - 1
        i += 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(prev, dtype=np.uint64))
    ref = [int(v) for v in bg.random_raw(4)]
    assert O.philox4x64(ctr, key) == ref


def test_uniform_open_interval():
    assert O.u01(0) == 2.0 ** -53
    assert O.u01(2**64 - 1) == 1.0 - 2.0 ** -53
    assert O.u01(2**63) == 0.5 + 2.0 ** -53


# --------------------------------------------------------------------------
# Potentials: closed forms and limits.
# --------------------------------------------------------------------------
def lj_params(**kw):
    p = W.lj_electrolyte(4, 0.1, 1).params
    p.update(kw)
    return p


def test_lj_closed_form_points():
    p = lj_params(charge=[0.0, 0.0])
    rc = p["rc_lj"]
    shift = 4.0 * ((1 / rc) ** 12 - (1 / rc) ** 6)
    # U(sigma) = -shift; minimum at 2^(1/6) sigma with depth -eps - shift
    ulj, uc, dlj, dc = O.pair(p, 0, 1, 1.0)
    assert ulj == pytest.approx(-shift, abs=1e-14)
    rmin = 2 ** (1 / 6)
    ulj, _, dlj, _ = O.pair(p, 0, 1, rmin)
    assert ulj == pytest.approx(-1.0 - shift, abs=1e-13)
    assert abs(dlj) < 1e-12
    # truncated: zero energy at and beyond the cutoff, force not shifted
    assert O.pair(p, 0, 1, rc)[0] == 0.0
    ulj, _, dlj, _ = O.pair(p, 0, 1, rc * (1 - 1e-12))
    assert abs(ulj) < 1e-10
    assert dlj == pytest.approx(4.0 * (-12 * rc ** -13 + 6 * rc ** -7), rel=1e-9)


def test_lorentz_berthelot_mixing():
    w = W.water_nacl(n_water=1, n_pairs=1, m=3, L=20.0)
    p = dict(w.params, charge=[0.0] * 4)
    # Na-Cl: sigma = (2.16 + 4.83)/2, eps = sqrt(0.35 * 0.0128): U(sigma_ij) = -shift_ij
    sig, eps = 0.5 * (2.16 + 4.83), math.sqrt(0.35 * 0.0128)
    shift = 4 * eps * ((sig / 10.0) ** 12 - (sig / 10.0) ** 6)
    assert O.pair(p, 2, 3, sig)[0] == pytest.approx(-shift, rel=1e-12)
    # hydrogens carry no Lennard-Jones site
    assert O.pair(p, 1, 2, 0.5)[0] == 0.0


@pytest.mark.parametrize("alpha,rc", [(0.3, 4.0), (0.25, 10.0)])
def test_dsf_vanishes_with_its_derivative_at_cutoff(alpha, rc):
    p = lj_params(eps=[0.0, 0.0], alpha=alpha, rc_coul=rc)
    for r in (rc * (1 - 1e-9), rc - 1e-7):
        _, uc, _, dc = O.pair(p, 0, 1, r)
        assert abs(uc) < 1e-9 and abs(dc) < 1e-6
    assert O.pair(p, 0, 1, rc)[1] == 0.0


def test_dsf_reduces_to_shifted_force_coulomb_without_damping():
    # alpha = 0: the textbook shifted-force Coulomb k q q (1/r - 1/Rc + (r - Rc)/Rc^2)
    p = lj_params(eps=[0.0, 0.0], alpha=0.0, rc_coul=4.0, coulomb_k=3.0)
    for r in (0.7, 1.3, 2.9):
        uc = O.pair(p, 0, 1, r)[1]
        assert uc == pytest.approx(3.0 * -1.0 * (1 / r - 1 / 4.0 + (r - 4.0) / 16.0), rel=1e-13)


def test_dsf_reduces_to_bare_and_screened_coulomb():
    # long cutoff: the shifts vanish; alpha -> 0 leaves bare Coulomb k q q / r,
    # finite alpha leaves the Ewald real-space kernel k q q erfc(alpha r)/r (scipy)
    p = lj_params(eps=[0.0, 0.0], alpha=1e-9, rc_coul=1e7, coulomb_k=3.0)
    for r in (0.8, 2.0, 5.0):
        assert O.pair(p, 0, 1, r)[1] == pytest.approx(-3.0 / r, rel=1e-6)
    p = lj_params(eps=[0.0, 0.0], alpha=0.3, rc_coul=200.0, coulomb_k=3.0)
    for r in (0.8, 2.0, 5.0):
        assert O.pair(p, 0, 0, r)[1] == pytest.approx(3.0 * erfc(0.3 * r) / r, rel=1e-9, abs=1e-12)


def test_dsf_force_shift_matches_library_erfc():
    # the force shift is minus the unshifted radial force at R_c
    for alpha, rc in [(0.3, 4.0), (0.25, 10.0)]:
        p = lj_params(eps=[0.0, 0.0], alpha=alpha, rc_coul=rc, coulomb_k=1.0)
        r = 1.7
        dc = O.pair(p, 0, 0, r)[3]
        sc = erfc(alpha * rc) / rc ** 2 + 2 * alpha / math.sqrt(math.pi) * math.exp(-(alpha * rc) ** 2) / rc
        unshifted = -erfc(alpha * r) / r ** 2 - 2 * alpha / math.sqrt(math.pi) * math.exp(-(alpha * r) ** 2) / r
        assert dc == pytest.approx(unshifted + sc, rel=1e-12)


def test_pair_derivatives_match_finite_differences():
    for params, ti, tj in [(lj_params(), 0, 1), (W.water_nacl(1, 1, m=3, L=20.0).params, 0, 2)]:
        for r in (0.95, 1.4, 2.2, 3.3) if params["n_types"] == 2 else (2.6, 4.0, 7.5, 9.5):
            h = 1e-6 * r
            up, um = O.pair(params, ti, tj, r + h), O.pair(params, ti, tj, r - h)
            d = O.pair(params, ti, tj, r)
            fd_lj = (up[0] - um[0]) / (2 * h)
            fd_c = (up[1] - um[1]) / (2 * h)
            assert d[2] == pytest.approx(fd_lj, rel=1e-6, abs=1e-9)
            assert d[3] == pytest.approx(fd_c, rel=1e-6, abs=1e-9)


# --------------------------------------------------------------------------
# Configurations: forces are minus the gradient, including the altitude.
# --------------------------------------------------------------------------
def small_system(n=24, rho=0.02, seed=3, flyers=(0, 1), kappa=0.0, **kw):
    w = W.lj_electrolyte(n, rho, seed)
    w.params.update(kappa_sr=kappa, **kw)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    for f in flyers:
        s.flying[f] = 1
    return s


@pytest.mark.parametrize("kappa", [0.0, 0.8])
def test_forces_are_minus_gradient_4d(kappa):
    s = small_system(kappa=kappa)
    w = 0.9
    e, F = s.compute(w)
    rng = np.random.default_rng(0)
    for i in rng.choice(s.n, 6, replace=False):
        for d in range(3):
            h = 1e-6
            x0 = s.x[i, d]
            s.x[i, d] = x0 + h
            ep, _ = s.compute(w, forces=False)
            s.x[i, d] = x0 - h
            em, _ = s.compute(w, forces=False)
            s.x[i, d] = x0
            fd = -(ep.U - em.U) / (2 * h)
            assert F[i, d] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    h = 1e-6
    ep, _ = s.compute(w + h, forces=False)
    em, _ = s.compute(w - h, forces=False)
    assert e.dUdw == pytest.approx((ep.U - em.U) / (2 * h), rel=1e-6, abs=1e-7)


def test_newton_third_law():
    s = small_system(n=200, rho=0.3, kappa=0.5)
    e, F = s.compute(0.7)
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()


def test_cell_search_equals_all_pairs():
    w = W.lj_electrolyte(600, 0.3, 5)   # L = 12.6: 3 cells of 4.2 per side
    a = O.OracleSystem.from_workload(w, use_cells=False)
    b = O.OracleSystem.from_workload(w, use_cells=True)
    for s in (a, b):
        s.flying[3] = s.flying[10] = 1
    ea, Fa = a.compute(1.1)
    eb, Fb = b.compute(1.1)
    assert eb.U == pytest.approx(ea.U, rel=1e-12)
    assert np.abs(Fa - Fb).max() < 1e-11


def test_four_d_distance_and_screening_of_a_single_pair():
    # one flyer above a non-flyer at 3D distance r: energy of the pair at
    # s = sqrt(r^2 + w^2), Coulomb times exp(-kappa w)
    p = lj_params(kappa_sr=0.7)
    L = 20.0
    p["box"] = [L, L, L]
    x = np.array([[5.0, 5.0, 5.0], [6.2, 5.0, 5.0]])
    s = O.OracleSystem(p, x, np.array([0, 1], np.int32), np.array([-1, -1], np.int32),
                       np.array([0, 1], np.int64), 1, use_cells=False)
    s.flying[0] = 1
    for w in (0.0, 0.5, 1.7, 3.0):
        e, _ = s.compute(w, forces=False)
        ulj, uc, _, _ = O.pair(p, 0, 1, math.hypot(1.2, w))
        assert e.U == pytest.approx(ulj + math.exp(-0.7 * w) * uc, rel=1e-13, abs=1e-15)
    # both flying: same altitude, so 3D distance and no screening
    s.flying[1] = 1
    e, _ = s.compute(2.0, forces=False)
    ulj, uc, _, _ = O.pair(p, 0, 1, 1.2)
    assert e.U == pytest.approx(ulj + uc, rel=1e-13)


# --------------------------------------------------------------------------
# Switching accounting in closed form.
# --------------------------------------------------------------------------
def test_lone_pair_insertion_energy_is_the_pair_energy():
    # an empty box: the whole dH of an insertion is the pair's own energy at
    # its 3D separation, all of it in the switch-on term, no protocol work
    w = W.ideal_gas(L=12.0, beta_mu=0.0, n_steps=5)
    w.params.update(charge=[1.0, -1.0], eps=[1.0, 1.0])
    s = O.OracleSystem.from_workload(w, use_cells=False)
    rec = s.trial(0, force_move=+1)
    # recover the ion positions the trial drew
    u = [O.u01(b) for b in O.philox4x64((0, 1, 0, 0), (w.params["seed"], 0))] + \
        [O.u01(b) for b in O.philox4x64((0, 1, 1, 0), (w.params["seed"], 0))]
    rc_, ra_ = 12.0 * np.array(u[1:4]), 12.0 * np.array(u[4:7])
    d = rc_ - ra_
    d -= 12.0 * np.round(d / 12.0)
    ulj, uc, _, _ = O.pair(w.params, 0, 1, float(np.linalg.norm(d)))
    assert rec["dH"] == pytest.approx(ulj + uc, rel=1e-12, abs=1e-14)
    assert rec["E_switch"] == pytest.approx(ulj + uc, rel=1e-12, abs=1e-14)
    assert rec["W_prot"] == 0.0


def test_protocol_work_telescopes_against_a_frozen_partner():
    # a flyer above an immobile partner: the protocol work is exactly
    # U(r; w_end) - U(r; w_start) (Eq. 2 schedule), and dH has no shadow part
    p = lj_params(kappa_sr=0.4, mass=[1.0, 1e300])
    L = 20.0
    p["box"] = [L, L, L]
    x = np.array([[5.0, 5.0, 5.0], [6.1, 5.3, 4.8]])
    s = O.OracleSystem(p, x, np.array([0, 1], np.int32), np.array([-1, -1], np.int32),
                       np.array([0, 1], np.int64), 1, use_cells=False)
    s.flying[0] = 1
    r = float(np.linalg.norm(x[1] - x[0]))
    wmax = p["w_max"]
    W_ = s.nemd(+1, 37)

    def U(w):
        ulj, uc, _, _ = O.pair(p, 0, 1, math.hypot(r, w))
        return ulj + math.exp(-0.4 * w) * uc
    assert W_ == pytest.approx(U(0.0) - U(wmax), rel=1e-12, abs=1e-14)


# --------------------------------------------------------------------------
# Integrator: second order, reversible, work = energy change as dt -> 0.
# --------------------------------------------------------------------------
def _nve_drift(dt, T_total=0.4):
    # like charges, no LJ: the damped shifted force is continuous at its
    # cutoff, so velocity Verlet's global energy error is O(dt^2) (the LJ of
    # Eq. 19 keeps a force jump at r_c that adds O(dt) per crossing)
    w = W.lj_electrolyte(200, 0.3, 9)
    w.params.update(dt=dt, charge=[1.0, 1.0], eps=[0.0, 0.0])
    s = O.OracleSystem.from_workload(w, use_cells=False)
    s.mb(3)
    e0, _ = s.compute()
    H0 = e0.U + s.kinetic()
    s.nemd(+1, int(round(T_total / dt)))
    e1, _ = s.compute()
    return abs(e1.U + s.kinetic() - H0)


def test_energy_error_is_second_order():
    d1, d2 = _nve_drift(0.004), _nve_drift(0.002)
    assert 2.5 < d1 / d2 < 6.0


def test_trajectory_is_time_reversible():
    s = small_system(n=200, rho=0.3, kappa=0.6)
    s.mb(1)
    x0 = s.positions()
    s.nemd(+1, 100)            # insertion schedule: w_max -> 0
    s.v *= -1.0
    s.nemd(-1, 100)            # the reversed schedule: 0 -> w_max
    d = s.positions() - x0
    d -= s.pd["box"][0] * np.round(d / s.pd["box"][0])
    assert np.abs(d).max() < 1e-9


def test_shadow_work_vanishes_as_dt_squared():
    # dH = E_switch + W_prot + S; at a fixed switching time N_f dt the shadow
    # part S shrinks like dt^2
    # continuous force (like charges, damped shifted force only, screened)
    out = []
    for nf in (100, 200):
        w = W.lj_electrolyte(200, 0.3, 13)
        w.params.update(dt=0.5 / nf, n_steps=nf, charge=[1.0, 1.0], eps=[0.0, 0.0], kappa_sr=0.5)
        s = O.OracleSystem.from_workload(w, use_cells=False)
        rec = s.trial(4, force_move=+1)
        out.append(rec["dH"] - rec["E_switch"] - rec["W_prot"])
    assert abs(out[0]) > 0
    assert 2.5 < abs(out[0]) / abs(out[1]) < 6.0


def test_metropolis_bookkeeping():
    w = W.lj_electrolyte(200, 0.3, 17, n_steps=10)
    w.params.update(beta_mu=-3.0)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    V = w.params["box"][0] ** 3
    for t in range(12):
        ns = s.nsalt
        rec = s.trial(t)
        nsmall = ns if rec["move"] > 0 else ns - 1
        I = 2 * math.log(V / (nsmall + 1))
        if rec["move"] > 0:
            assert rec["ln_ratio"] == pytest.approx(-rec["dH"] - 3.0 + I, rel=1e-12)
            assert rec["dM"] == pytest.approx(rec["dH"] - I, rel=1e-12)
            assert rec["ln_ratio"] == pytest.approx(-(rec["dM"] - (-3.0)), rel=1e-12)
        else:
            assert rec["ln_ratio"] == pytest.approx(-rec["dH"] + 3.0 - I, rel=1e-12)
            assert rec["ln_ratio"] == pytest.approx(rec["dM"] - (-3.0), rel=1e-12)
        assert rec["accepted"] == int(rec["ln_u"] < rec["ln_ratio"])
        assert s.nsalt == ns + rec["accepted"] * rec["move"]
        assert s.n == 2 * s.nsalt


# --------------------------------------------------------------------------
# The acceptance rule is exact: ideal ion pairs reach P(N) ~ y^(2N)/(N!)^2.
# --------------------------------------------------------------------------
def ideal_closed_form(y, nmax=200):
    n = np.arange(nmax)
    logp = 2 * n * math.log(y) - 2 * np.array([math.lgamma(k + 1) for k in n])
    p = np.exp(logp - logp.max())
    return p / p.sum()


def test_ideal_closed_form_moments():
    gold = json.load(open(os.path.join(GOLD, "ideal_limit.json")))
    for y in (10.0, 250.0):
        p = ideal_closed_form(y, 2000)
        n = np.arange(len(p))
        mean = (p * n).sum()
        var = (p * n * n).sum() - mean ** 2
        assert mean == pytest.approx(y * i1(2 * y) / i0(2 * y) if y < 300 else mean, rel=1e-10)
        chi = var / mean
        assert abs(chi - gold["chi_osmotic_ideal"]) < (0.02 if y == 10.0 else 0.001)


def test_ideal_reservoir_stationary_distribution():
    y, L = 3.0, 5.0
    beta_mu = 2 * math.log(y / L ** 3)
    w = W.ideal_gas(L=L, beta_mu=beta_mu, n_steps=1)
    s = O.OracleSystem.from_workload(w, cap=256, use_cells=False)
    ns = []
    for t in range(60000):
        s.trial(t)
        ns.append(s.nsalt)
    ns = np.array(ns[1000:])
    exact = ideal_closed_form(y, 60)
    emp = np.bincount(ns, minlength=60)[:60] / len(ns)
    assert 0.5 * np.abs(emp - exact).sum() < 0.02
    mean_exact = y * i1(2 * y) / i0(2 * y)
    assert ns.mean() == pytest.approx(mean_exact, abs=0.06)


def _altitudes(schedule, n, move, nf=50, w_max=2.5):
    p = O.make_params(dict(W.lj_electrolyte(24, 0.02, 3).params, schedule=schedule, schedule_n=n, w_max=w_max))
    return np.array([O.lib().or_altitude(ctypes.byref(p), move, k, nf) for k in range(nf + 1)])


@pytest.mark.parametrize("schedule", [1, 2])
def test_variable_velocity_schedules(schedule):
    # the supplement's w_v (1) and w_x (2): endpoints w_max and 0, n = 1 is
    # Eq. (2), and the deletion runs the insertion's schedule backwards
    ins = _altitudes(schedule, 3.0, +1)
    dele = _altitudes(schedule, 3.0, -1)
    assert ins[0] == pytest.approx(2.5, abs=1e-15) and ins[-1] == pytest.approx(0.0, abs=1e-15)
    assert np.allclose(dele, ins[::-1], rtol=0, atol=1e-15)
    assert np.allclose(_altitudes(schedule, 1.0, +1), _altitudes(0, 1.0, +1), rtol=0, atol=1e-14)
    x = 0.5
    mid = ins[25]
    # w_v is slow near w_max first (concave), w_x fast first (convex)
    assert mid == pytest.approx(2.5 * ((1 - x ** 3) if schedule == 1 else (1 - x) ** 3), rel=1e-14)
    assert (mid > 2.5 * 0.5) == (schedule == 1)


@pytest.mark.parametrize("schedule", [1, 2])
def test_trajectory_is_time_reversible_with_a_variable_schedule(schedule):
    # with the deletion the time reversal of the insertion's schedule, the
    # reversed NEMD returns to the start (the deletion formulas as printed
    # pair w_v's insertion with w_x's reversal and would not)
    s = small_system(n=200, rho=0.3, kappa=0.6, schedule=schedule, schedule_n=2.5)
    s.mb(1)
    x0 = s.positions()
    s.nemd(+1, 100)
    s.v *= -1.0
    s.nemd(-1, 100)
    d = s.positions() - x0
    d -= s.pd["box"][0] * np.round(d / s.pd["box"][0])
    assert np.abs(d).max() < 1e-9
