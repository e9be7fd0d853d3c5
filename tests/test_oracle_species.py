"""Pins of species-specific w_max (the supplement's remedy for overlapping
flyers): the anion flies at r_w times the cation's altitude, both reach
w = 0 together, flyer-flyer pairs see (w_c - w_a)^2, and Eq. 11 screening
uses the flyers' mean altitude."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def lj_params(**kw):
    p = W._base_lj_params(20.0)
    p.update(kw)
    return p


def two_ions(p, flying, x=((5.0, 5.0, 5.0), (6.2, 5.0, 5.0))):
    s = O.OracleSystem(p, np.array(x), np.array([0, 1], np.int32), np.array([-1, -1], np.int32),
                       np.array([0, 1], np.int64), 1, use_cells=False)
    for f in flying:
        s.flying[f] = 1
    return s


@pytest.mark.parametrize("ratio", [1.6, 0.7])
def test_one_flyer_sits_at_its_own_altitude_and_screening_at_the_mean(ratio):
    p = lj_params(kappa_sr=0.7, w_max_ratio=ratio)
    for w in (0.0, 0.5, 1.7):
        # the anion (type 1) flies above the cation: its altitude is ratio * w
        e, _ = two_ions(p, [1]).compute(w, forces=False)
        ulj, uc, _, _ = O.pair(p, 0, 1, math.hypot(1.2, ratio * w))
        assert e.U == pytest.approx(ulj + math.exp(-0.7 * 0.5 * w * (1 + ratio)) * uc, rel=1e-13, abs=1e-15)
        # the cation flies: its altitude is w
        e, _ = two_ions(p, [0]).compute(w, forces=False)
        ulj, uc, _, _ = O.pair(p, 0, 1, math.hypot(1.2, w))
        assert e.U == pytest.approx(ulj + math.exp(-0.7 * 0.5 * w * (1 + ratio)) * uc, rel=1e-13, abs=1e-15)
        # both fly: 4D distance with (w_c - w_a)^2, unscreened
        e, _ = two_ions(p, [0, 1]).compute(w, forces=False)
        ulj, uc, _, _ = O.pair(p, 0, 1, math.hypot(1.2, (1 - ratio) * w))
        assert e.U == pytest.approx(ulj + uc, rel=1e-13, abs=1e-15)


def test_ratio_one_and_zero_are_the_common_altitude():
    w = W.lj_electrolyte(200, 0.3, 8)
    out = []
    for ratio in (0.0, 1.0):
        s = O.OracleSystem(dict(w.params, kappa_sr=0.4, w_max_ratio=ratio), w.x, w.type, w.mol, w.tag, w.nsalt,
                           use_cells=False)
        s.flying[int(np.flatnonzero(w.type == 0)[0])] = 1
        s.flying[int(np.flatnonzero(w.type == 1)[0])] = 1
        out.append(s.compute(1.3)[0].U)
    assert out[0] == out[1]


@pytest.mark.parametrize("ratio", [1.8, 0.6])
def test_forces_and_altitude_derivative_with_species_altitudes(ratio):
    w = W.lj_electrolyte(24, 0.02, 3)
    w.params.update(kappa_sr=0.8, w_max_ratio=ratio)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    ic = int(np.flatnonzero(w.type == 0)[0])
    ia = int(np.flatnonzero(w.type == 1)[0])
    s.flying[ic] = s.flying[ia] = 1
    # bring the flyers close together so that their own pair is in range
    s.x[ia] = s.x[ic] + np.array([1.1, 0.2, -0.3])
    wv = 0.9
    e, F = s.compute(wv)
    h = 1e-6
    for i in range(s.n):
        if s.flying[i]:
            continue
        for d in range(3):
            x0 = s.x[i, d]
            s.x[i, d] = x0 + h
            ep, _ = s.compute(wv, forces=False)
            s.x[i, d] = x0 - h
            em, _ = s.compute(wv, forces=False)
            s.x[i, d] = x0
            assert F[i, d] == pytest.approx(-(ep.U - em.U) / (2 * h), rel=1e-6, abs=1e-7)
    ep, _ = s.compute(wv + h, forces=False)
    em, _ = s.compute(wv - h, forces=False)
    assert e.dUdw == pytest.approx((ep.U - em.U) / (2 * h), rel=1e-6, abs=1e-7)


@pytest.mark.parametrize("ratio", [1.5, 0.8])
def test_lone_pair_insertion_with_species_altitudes(ratio):
    # an empty box: dH of an insertion is the pair's energy at its 3D
    # separation; the switch-on term is the pair at (1 - r_w) w_max above
    # each other and the protocol work the rest (it telescopes: flyers stay
    # fixed in 3D)
    w = W.ideal_gas(L=12.0, beta_mu=0.0, n_steps=7)
    w.params.update(charge=[1.0, -1.0], eps=[1.0, 1.0], w_max_ratio=ratio)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    rec = s.trial(0, force_move=+1)
    u = [O.u01(b) for b in O.philox4x64((0, 1, 0, 0), (w.params["seed"], 0))] + \
        [O.u01(b) for b in O.philox4x64((0, 1, 1, 0), (w.params["seed"], 0))]
    d = 12.0 * np.array(u[1:4]) - 12.0 * np.array(u[4:7])
    d -= 12.0 * np.round(d / 12.0)
    r = float(np.linalg.norm(d))
    wmax = w.params["w_max"]

    def U(x):
        ulj, uc, _, _ = O.pair(w.params, 0, 1, x)
        return ulj + uc
    assert rec["dH"] == pytest.approx(U(r), rel=1e-12, abs=1e-14)
    assert rec["E_switch"] == pytest.approx(U(math.hypot(r, (1 - ratio) * wmax)), rel=1e-12, abs=1e-14)
    assert rec["W_prot"] == pytest.approx(U(r) - rec["E_switch"], rel=1e-10, abs=1e-12)


def test_trajectory_is_time_reversible_with_species_altitudes():
    w = W.lj_electrolyte(200, 0.3, 11)
    w.params.update(kappa_sr=0.6, w_max_ratio=1.7)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    s.flying[int(np.flatnonzero(w.type == 0)[0])] = 1
    s.flying[int(np.flatnonzero(w.type == 1)[0])] = 1
    s.mb(1)
    x0 = s.positions()
    s.nemd(+1, 100)
    s.v *= -1.0
    s.nemd(-1, 100)
    d = s.positions() - x0
    d -= s.pd["box"][0] * np.round(d / s.pd["box"][0])
    assert np.abs(d).max() < 1e-9
