"""Pins of the oracle's rigid-water treatment: the bond constraints hold
after every step, constrained velocities have no component along any bond,
the trajectory is time reversible, constrained Maxwell-Boltzmann momenta
carry kT/2 per remaining degree of freedom, and intramolecular pairs are
excluded from the energy."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def small_water(n_water=60, n_pairs=2, L=14.5, m=6, seed=5, rc=6.0):
    w = W.water_nacl(n_water=n_water, n_pairs=n_pairs, L=L, m=m, seed=seed)
    w.params.update(rc_lj=rc, rc_coul=rc, n_steps=20)
    return w


def bond_errors(s, p):
    L = p["box"][0]
    errs = []
    for k in range(s.s.n_mol):
        o, h1, h2 = 3 * k, 3 * k + 1, 3 * k + 2
        for a, b, d in ((o, h1, p["d_oh"]), (o, h2, p["d_oh"]), (h1, h2, p["d_hh"])):
            r = s.x[a] - s.x[b]
            r -= L * np.round(r / L)
            errs.append(abs(np.linalg.norm(r) - d) / d)
    return max(errs)


def bond_velocity_errors(s, p):
    L = p["box"][0]
    worst = 0.0
    for k in range(s.s.n_mol):
        o, h1, h2 = 3 * k, 3 * k + 1, 3 * k + 2
        for a, b in ((o, h1), (o, h2), (h1, h2)):
            r = s.x[a] - s.x[b]
            r -= L * np.round(r / L)
            dv = s.v[a] - s.v[b]
            worst = max(worst, abs(r @ dv) / (np.linalg.norm(r) * (np.linalg.norm(dv) + 1e-30)))
    return worst


def test_constraints_hold_along_a_trajectory():
    w = small_water()
    s = O.OracleSystem.from_workload(w, use_cells=False)
    assert bond_errors(s, w.params) < 1e-12
    s.mb(1)
    assert bond_velocity_errors(s, w.params) < 1e-10
    s.nemd(+1, 20)
    assert bond_errors(s, w.params) < 1e-12
    assert bond_velocity_errors(s, w.params) < 1e-10


def test_water_trajectory_is_time_reversible():
    w = small_water()
    s = O.OracleSystem.from_workload(w, use_cells=False)
    s.flying[3 * 60] = 1   # one ion flying
    s.mb(2)
    x0 = s.positions()
    s.nemd(+1, 30)
    s.v *= -1.0
    s.nemd(-1, 30)
    d = s.positions() - x0
    L = w.params["box"][0]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-8


def test_constrained_momenta_have_kT_over_2_per_degree_of_freedom():
    w = small_water(n_water=60, n_pairs=2)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    kT = w.params["kT"]
    dof = 6 * 60 + 3 * 4          # rigid waters: 6 each; ions: 3 each
    Ks = []
    for t in range(200):
        s.mb(t)
        Ks.append(s.kinetic())
    mean = np.mean(Ks)
    # K ~ (kT/2) chi^2_dof: mean dof kT/2, sd kT sqrt(dof/2); 200 samples
    assert abs(mean - 0.5 * dof * kT) < 4 * kT * math.sqrt(dof / 2) / math.sqrt(200)


def test_intramolecular_pairs_are_excluded():
    # one isolated water: its energy is zero whatever its charges and geometry
    w = W.water_nacl(n_water=1, n_pairs=0, L=14.0, m=3, seed=1)
    w.params.update(rc_lj=6.0, rc_coul=6.0)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    e, F = s.compute(0.0)
    assert e.U == 0.0 and np.abs(F).max() == 0.0
