"""Pins of early rejection (the supplement's instantaneous exchange of a pair
in contact): a pair whose anion lies in the cube V_ex centred on the cation
is exchanged with no trajectory, for insertions and deletions alike."""
import math

import numpy as np
import pytest
from scipy.special import i0, i1

from oracle import oracle as O
from paper_2307_11447_amd import workloads as W


def drawn_pair(params, t, L):
    u = [O.u01(b) for b in O.philox4x64((t, 1, 0, 0), (params["seed"], params.get("stream", 0)))] + \
        [O.u01(b) for b in O.philox4x64((t, 1, 1, 0), (params["seed"], params.get("stream", 0)))]
    return L * np.array(u[1:4]), L * np.array(u[4:7])


def inside(xc, xa, L, edge):
    d = xa - xc
    d -= L * np.round(d / L)
    return bool(np.all(np.abs(d) < 0.5 * edge))


def test_instant_insertion_is_the_energy_difference_of_the_two_states():
    w = W.lj_electrolyte(40, 0.04, 12, n_steps=10)
    L = w.params["box"][0]
    w.params.update(v_ex_edge=4.0, beta_mu=-1000.0)
    s = O.OracleSystem.from_workload(w, cap=w.n + 8, use_cells=False)
    e0, _ = s.compute(0.0, forces=False)
    n_inst = 0
    for t in range(300):
        r = s.trial(t, +1)
        xc, xa = drawn_pair(w.params, t, L)
        assert bool(r["flags"] & O.FLAG_INSTANT) == inside(xc, xa, L, 4.0)
        if not r["flags"] & O.FLAG_INSTANT:
            continue
        n_inst += 1
        assert r["n_steps"] == 0 and r["dK"] == 0.0 and r["W_prot"] == 0.0
        # the (N+1)-state with the pair in 3D, built independently
        x = np.vstack([w.x, np.mod(xc, L), np.mod(xa, L)])
        t_ = np.concatenate([w.type, [0, 1]]).astype(np.int32)
        big = O.OracleSystem(w.params, x, t_, np.full(w.n + 2, -1, np.int32), np.arange(w.n + 2, dtype=np.int64),
                             w.nsalt + 1, use_cells=False)
        e1, _ = big.compute(0.0, forces=False)
        assert r["dH"] == pytest.approx(e1.U - e0.U, rel=1e-10, abs=1e-10)
    assert n_inst > 10


def test_share_of_instant_insertions_is_v_ex_over_v():
    L, edge = 5.0, 2.0
    w = W.ideal_gas(L=L, beta_mu=-1000.0, n_steps=1)
    w.params.update(v_ex_edge=edge)
    s = O.OracleSystem.from_workload(w, cap=16, use_cells=False)
    n = 4000
    k = sum(bool(s.trial(t, +1)["flags"] & O.FLAG_INSTANT) for t in range(n))
    p = edge ** 3 / L ** 3
    assert abs(k / n - p) < 4.0 * math.sqrt(p * (1 - p) / n)


def test_deletion_takes_the_type_of_its_pair():
    w = W.lj_electrolyte(120, 0.1, 14, n_steps=5)
    L = w.params["box"][0]
    w.params.update(v_ex_edge=3.5, beta_mu=1000.0)
    s = O.OracleSystem.from_workload(w, use_cells=False)
    pos = {int(g): w.x[q] for q, g in enumerate(w.tag)}
    seen = set()
    for t in range(200):
        r = s.trial(t, -1)
        xc, xa = pos[r["tag_c"]], pos[r["tag_a"]]
        flag = bool(r["flags"] & O.FLAG_INSTANT)
        assert flag == inside(xc, xa, L, 3.5)
        assert (r["n_steps"] == 0) == flag
        seen.add(flag)
    assert seen == {False, True}


def test_ideal_reservoir_with_early_rejection():
    y, L = 3.0, 5.0
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    w.params.update(v_ex_edge=2.5)
    s = O.OracleSystem.from_workload(w, cap=256, use_cells=False)
    ns = []
    for t in range(40000):
        s.trial(t)
        ns.append(s.nsalt)
    ns = np.array(ns[1000:])
    assert ns.mean() == pytest.approx(y * i1(2 * y) / i0(2 * y), abs=0.08)


def _gc_mean_n(edge, n, seed=5):
    w = W.lj_electrolyte(20, 0.02, seed, n_steps=10)
    w.params.update(beta_mu=-10.5, dt=0.01, v_ex_edge=edge)
    s = O.OracleSystem.from_workload(w, cap=400, use_cells=False)
    N = []
    for t in range(n):
        s.trial(t)
        N.append(s.nsalt)
    N = np.array(N[1000:], dtype=float)
    nb = 25
    b = N[: len(N) // nb * nb].reshape(nb, -1).mean(1)
    return N.mean(), b.std(ddof=1) / math.sqrt(nb)


def test_early_rejection_samples_the_same_reservoir():
    m0, e0 = _gc_mean_n(0.0, 16000)
    m1, e1 = _gc_mean_n(5.0, 16000)
    assert abs(m0 - m1) < 4.0 * math.hypot(e0, e1) + 0.05
