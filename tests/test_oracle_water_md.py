"""Pins of the oracle's equilibrium phase with rigid waters (generalized
hybrid MC with constraints, the phase between trials of Sec. II A, Fig. 1)
and of trials that carry rigid waters' momenta.

- the phase's constrained velocity Verlet (SHAKE positions, RATTLE
  velocities) conserves H to second order in dt;
- after every phase and every carried-momentum trial the positions meet the
  constraints and the momenta have no bond component;
- the refreshed momenta carry kT/2 per degree of freedom the constraints
  leave (3 N - 3 n_mol in all), not per Cartesian one;
- a rejected phase keeps the positions and reverses the refreshed momenta;
- phases and carried-momentum trials alternate as the cycle of Fig. 1 does.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def small_water(seed=78, **kw):
    w = W.water_nacl(n_water=300, n_pairs=10, L=21.0, m=7, seed=seed)
    w.params.update(precision="fp64", **kw)
    return w


def bond_checks(o, w):
    """Worst relative constraint error of the positions and worst bond
    component of the velocities (relative to |v| |r|)."""
    p = w.params
    L = p["box"][0]
    x, v = o.positions(), o.velocities()
    pos_err = vel_err = 0.0
    for m in range(w.n_mol):
        a0 = 3 * m
        for (i, j, d) in ((a0, a0 + 1, p["d_oh"]), (a0, a0 + 2, p["d_oh"]), (a0 + 1, a0 + 2, p["d_hh"])):
            r = x[i] - x[j]
            r -= L * np.round(r / L)
            dv = v[i] - v[j]
            pos_err = max(pos_err, abs(np.linalg.norm(r) - d) / d)
            vel_err = max(vel_err, abs(dv @ r) / (np.linalg.norm(r) * max(np.linalg.norm(dv), 1e-300)))
    return pos_err, vel_err


def test_water_phase_energy_error_is_second_order():
    # no LJ (the truncated LJ force jumps at the cutoff); DSF Coulomb's force
    # is continuous there, so the error is the integrator's own
    def dH(dt):
        w = small_water(dt=dt, eps=[0.0, 0.0, 0.0, 0.0], md_refresh=0.0)
        o = O.OracleSystem.from_workload(w, use_cells=False)
        return abs(o.md_phase(5, int(round(16.0 / dt)))["dH"])
    d1, d2 = dH(1.0), dH(0.5)
    assert 2.5 < d1 / d2 < 6.0


def test_water_phase_keeps_constraints_and_equipartition():
    w = small_water(dt=1.0, md_refresh=0.0)
    beta = 1.0 / w.params["kT"]
    o = O.OracleSystem.from_workload(w, use_cells=False)
    assert max(bond_checks(o, w)) < 1e-10              # the set-up momenta are restricted too
    dof = 3 * w.n - 3 * w.n_mol
    ks = []
    for t in range(24):
        e, _ = o.compute(0.0, forces=False)
        r = o.md_phase(t, 4)
        ks.append(beta * (r["H0"] - e.U))                 # the refreshed momenta's K (c = 0: a fresh draw)
        pe, ve = bond_checks(o, w)
        assert pe < 1e-10 and ve < 1e-9, (t, pe, ve)
    ratio = np.mean(ks) / (0.5 * dof)
    # 24 independent draws of a chi-square with 1890 degrees of freedom: the
    # mean lies within 1 % of dof / 2; a refresh left on all 3 N Cartesian
    # components would give 3 N / dof = 1.48
    assert abs(ratio - 1.0) < 0.015, ratio


def test_rejected_water_phase_reverses_the_refreshed_momenta():
    c = 0.4
    w = small_water(dt=3.0, md_refresh=c)
    o = O.OracleSystem.from_workload(w, use_cells=False)
    seen = {0: 0, 1: 0}
    for t in range(16):
        x0, v0 = o.positions(), o.velocities()
        r = o.md_phase(t, 12)
        seen[r["accepted"]] += 1
        if not r["accepted"]:
            assert np.array_equal(o.positions(), x0)
            # -v = c v0 + sqrt(1 - c^2) xi with xi restricted, so xi is tangent too
            xi = (-o.velocities() - c * v0) / np.sqrt(1 - c * c)
            m = np.array(w.params["mass"])[w.type]
            ke = 0.5 * np.sum(m[:, None] * xi * xi) / w.params["accel"]
            dof = 3 * w.n - 3 * w.n_mol
            assert abs(ke / (0.5 * dof * w.params["kT"]) - 1.0) < 0.15
        assert max(bond_checks(o, w)) < 1e-9
    assert seen[0] >= 2 and seen[1] >= 2, seen


def test_water_cycle_of_phases_and_carried_momentum_trials():
    w = small_water(dt=1.0, n_steps=15, momenta=1, md_refresh=0.5, beta_mu=-250.0)
    o = O.OracleSystem.from_workload(w, cap=w.n + 40, use_cells=False)
    acc = 0
    for t in range(6):
        o.md_phase(t, 5)
        x0, v0, n0 = o.positions(), o.velocities(), o.n
        r = o.trial(t)
        acc += r["accepted"]
        pe, ve = bond_checks(o, w)
        assert pe < 1e-10 and ve < 1e-9, (t, pe, ve)
        if not r["accepted"] and not r["flags"]:
            # a rejected trial: the start positions, every momentum times one sign
            assert o.n == n0 and np.array_equal(o.positions(), x0)
            sgn = np.sign(np.sum(o.velocities() * v0))
            assert np.allclose(o.velocities(), sgn * v0, rtol=0, atol=1e-12)
    assert acc >= 1
