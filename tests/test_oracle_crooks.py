"""Crooks' relation on the oracle's own trials: insertion and deletion work
sampled from equilibrium states (equilibrium phases between forced moves
that are never accepted) give one chemical potential whatever the speed of
the protocol; BAR agrees with the exponential (Jarzynski) average of the
deletions, and the second law orders the mean works around it.  These are
consistency checks of the trial's work (Eqs. 6 and 8) with the equilibrium
phase and the BAR solver (the supplement's CFT/BAR section), facts that hold
for any correct nonequilibrium protocol; at 600 samples they are too weak to
catch a faulty integrator, which the second-order and time-reversal pins
catch."""
import math

import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import oracle as O
from paper_2307_11447_amd import analysis as A
from paper_2307_11447_amd import workloads as W


def works(n_atoms, move, nf, n, seed, L=10.0):
    # an electrolyte of n_atoms in a box of edge L, equilibrated and then
    # sampled by generalized hybrid MC phases between forced moves
    w = W.lj_electrolyte(n_atoms, n_atoms / L ** 3, seed, n_steps=nf)
    w.params.update(dt=0.01, md_refresh=0.0, beta_mu=-1000.0 if move > 0 else 1000.0)
    s = O.OracleSystem.from_workload(w, cap=n_atoms + 8, use_cells=False)
    for t in range(50):
        s.md_phase(100000 + t, 20)
    out = []
    for t in range(n):
        s.md_phase(t, 10)
        r = s.trial(t, move)
        assert not r["accepted"]
        if not r["flags"]:
            out.append(r["dM"])
    return np.array(out)


@pytest.fixture(scope="module")
def samples():
    # 10 pairs -> 11 pairs: insertions on the 20-ion state, deletions on the 22-ion state
    return {nf: (works(20, +1, nf, 600, 3), works(22, -1, nf, 600, 4)) for nf in (5, 40)}


def test_bar_does_not_depend_on_the_protocol_speed(samples):
    mu = {nf: A.bar_beta_mu(i, d, 1.0) for nf, (i, d) in samples.items()}
    assert abs(mu[5] - mu[40]) < 0.3


def test_bar_agrees_with_the_exponential_average_of_deletions(samples):
    for ins, dele in samples.values():
        mu = A.bar_beta_mu(ins, dele, 1.0)
        jarzynski_del = logsumexp(dele) - math.log(len(dele))      # ln <exp(beta dM_del)> = beta mu
        assert mu == pytest.approx(jarzynski_del, abs=0.3)


def test_second_law_orders_the_mean_works(samples):
    for ins, dele in samples.values():
        mu = A.bar_beta_mu(ins, dele, 1.0)
        assert np.mean(dele) < mu < np.mean(ins)
