"""GPU parity: the HIP library against the FP64 CPU oracle on the same
seeded inputs, through the C ABI.

Tolerances:
* forces from identical states: FP64 mode 1e-12 relative; FP32 mode
  ||dF||_2 / ||F||_2 <= 1e-5 and |dF_i| <= 1e-5 max(|F_i|, F_rms) per atom,
  where an atom with a pair within 1e-6 of the Lennard-Jones cutoff (the
  force jumps there, and the FP32 distance decides whether the pair counts)
  may match the oracle with or without that pair;
* FP64 energies: 1e-12 relative;
* FP64 trials: identical accept/reject sequence, dH, W_prot and E_switch
  within 1e-6 relative (floor 1 kT);
* FP32 trials run in lockstep (the oracle restarts from the GPU's state
  every trial): identical decisions except near-ties.
"""
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


def pick_flyers(w):
    c = int(np.where(w.type == w.params["cation_type"])[0][3])
    a = int(np.where(w.type == w.params["anion_type"])[0][5])
    return c, a


def oracle_forces(w, flyers, wv, use_cells=True):
    s = O.OracleSystem.from_workload(w, use_cells=use_cells)
    for f in flyers:
        if f >= 0:
            s.flying[f] = 1
    e, F = s.compute(wv)
    return e, F


def cutoff_edge_terms(w, flyers, wv, eps=1e-6):
    """Pairs whose (4D) distance lies within eps of the Lennard-Jones cutoff,
    where the truncated-shifted potential's force jumps: whether such a pair
    counts is decided by the precision of the distance (FP32 on the GPU,
    FP64 in the oracle), and both outcomes are valid.  Returns, per atom, the
    force those pairs contribute (FP64, from the oracle's pair function)."""
    from scipy.spatial import cKDTree
    p = w.params
    L = p["box"][0]
    rc = p["rc_lj"]
    fly = np.zeros(w.n, bool)
    for f in flyers:
        if f >= 0:
            fly[f] = True
    tree = cKDTree(np.mod(w.x, L), boxsize=L)
    pairs = tree.query_pairs(rc + 1e-3, output_type="ndarray")
    extra = np.zeros((w.n, 3))
    for i, j in pairs:
        d = w.x[i] - w.x[j]
        d -= L * np.round(d / L)
        r2 = float(d @ d)
        s2 = r2 + (wv * wv if fly[i] != fly[j] else 0.0)
        if abs(math.sqrt(s2) - rc) > eps:
            continue
        ulj, uc, dlj, dc = O.pair(p, int(w.type[i]), int(w.type[j]), math.sqrt(s2) * (1 - 1e-12))
        f = -dlj / math.sqrt(s2) * d          # force on i from the LJ term
        extra[i] += f
        extra[j] -= f
    return extra


def compare_forces(Fg, Fr, mask, tol_rel, per_atom, edge=None):
    if edge is not None:
        # atoms with a pair at the cutoff: either outcome of the inclusion test is valid
        alt = Fr - edge
        use_alt = np.linalg.norm(Fg - alt, axis=1) < np.linalg.norm(Fg - Fr, axis=1)
        Fr = np.where(use_alt[:, None], alt, Fr)
    d = (Fg - Fr)[mask]
    ref = Fr[mask]
    rel = np.linalg.norm(d) / np.linalg.norm(ref)
    fmag = np.linalg.norm(ref, axis=1)
    frms = math.sqrt((fmag ** 2).mean())
    worst = (np.linalg.norm(d, axis=1) / np.maximum(fmag, frms)).max()
    say(f"   force rel l2 {rel:.3e}, worst per-atom {worst:.3e}")
    assert rel <= tol_rel
    assert worst <= per_atom


@pytest.mark.parametrize("n,prec,kappa", [
    (500, "fp64", 0.0), (500, "fp64", 0.7), (1000, "fp64", 0.5),
    (500, "fp32", 0.0), (1000, "fp32", 0.5), (4000, "fp32", 0.3),
])
def test_forces_match_oracle(n, prec, kappa):
    say(f"case forces n={n} prec={prec} kappa={kappa}")
    w = W.lj_electrolyte(n, 0.3, 100 + n, precision=prec)
    w.params.update(kappa_sr=kappa)
    flyers = pick_flyers(w)
    wv = 1.3
    sys_ = h4d.System.from_workload(w)
    Fg, eg = sys_.forces_at(flyers, wv)
    er, Fr = oracle_forces(w, flyers, wv)
    mask = np.ones(n, bool)
    mask[list(flyers)] = False
    if prec == "fp64":
        compare_forces(Fg, Fr, mask, 1e-12, 1e-11)
    else:
        compare_forces(Fg, Fr, mask, 1e-5, 1e-5, cutoff_edge_terms(w, flyers, wv))
    # FP64 energies in both modes
    assert eg["U"] == pytest.approx(er.U, rel=1e-12)
    assert eg["U_lj"] == pytest.approx(er.U_lj, rel=1e-12)
    assert eg["U_c"] == pytest.approx(er.U_c, rel=1e-12)
    assert np.all(Fg[~mask] == 0.0)
    sys_.close()


def test_forces_full_size_32k_fp32():
    say("case forces n=32000 fp32 (benchmark launch configuration)")
    w = W.config_lj_32k()
    w.params.update(kappa_sr=0.5)
    flyers = pick_flyers(w)
    sys_ = h4d.System.from_workload(w)
    Fg, eg = sys_.forces_at(flyers, 0.8)
    er, Fr = oracle_forces(w, flyers, 0.8)
    mask = np.ones(w.n, bool)
    mask[list(flyers)] = False
    edge = cutoff_edge_terms(w, flyers, 0.8)
    say(f"   {int((np.linalg.norm(edge, axis=1) > 0).sum())} atoms with a pair within 1e-6 of the LJ cutoff")
    compare_forces(Fg, Fr, mask, 1e-5, 1e-5, edge)
    assert eg["U"] == pytest.approx(er.U, rel=1e-12)
    sys_.close()


def test_no_flyer_forces_and_observables():
    say("case observables n=1000 fp64")
    w = W.lj_electrolyte(1000, 0.3, 5, precision="fp64")
    sys_ = h4d.System.from_workload(w)
    Fg, eg = sys_.forces_at((-1, -1), 0.0)
    er, Fr = oracle_forces(w, (), 0.0)
    compare_forces(Fg, Fr, np.ones(w.n, bool), 1e-12, 1e-11)
    obs = sys_.observables()
    assert obs["U"] == pytest.approx(er.U, rel=1e-12)
    assert obs["virial"] == pytest.approx(er.virial, rel=1e-11)
    assert obs["n_atoms"] == 1000 and obs["n_salt"] == 500
    sys_.close()


def rel_close(a, b, tol, floor=1.0):
    return abs(a - b) <= tol * max(abs(b), floor)


def test_fp64_trials_match_oracle_sequence():
    say("case trials lj500 fp64 (first configuration)")
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 400)
    n_acc = 0
    for t in range(40):
        rg = g.trial()
        ro = o.trial(t)
        assert rg["trial"] == t
        assert rg["move"] == ro["move"]
        assert rg["flags"] & 0x3 == ro["flags"]
        assert rg["tag_c"] == ro["tag_c"] or ro["flags"] & 1
        if not ro["flags"]:
            for key in ("dH", "W_prot", "E_switch", "dM", "H0", "H1"):
                assert rel_close(rg[key], ro[key], 1e-6), (t, key, rg[key], ro[key])
            assert rg["ln_ratio"] == pytest.approx(ro["ln_ratio"], rel=1e-6, abs=1e-6)
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        assert rg["n_salt_after"] == ro["n_salt_after"]
        n_acc += rg["accepted"]
    say(f"   accepted {n_acc} of 40")
    st = g.state()
    assert st["n"] == o.n
    assert np.array_equal(st["tag"], o.tag[: o.n])
    d = st["x"] - o.x[: o.n]
    L = w.params["box"][0]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-8
    g.close()


def test_autotuned_handle_matches_oracle():
    """The autotuner picks lanes per atom and the base rebuild interval by
    timing ordinary trials; the trials after it still follow the oracle
    (FP64, the same tolerances as the untuned sequence)."""
    say("case autotune lj500 fp64, then 12 trials against the oracle")
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0)
    g = h4d.System.from_workload(w)
    lanes, every, ns = g.autotune(1)
    say(f"   autotune: {lanes} lanes per atom, rebuild every {every} steps, {ns:.3f} ns per atom-step")
    assert lanes in (4, 8, 16) and every >= 1 and ns > 0.0
    st = g.state()
    o = O.OracleSystem(w.params, st["x"], st["type"], st["mol"], st["tag"], st["nsalt"], cap=st["n"] + 200)
    rg = g.trial()
    t0 = rg["trial"]
    assert t0 >= 8                   # 3 lane choices and at least 1 interval, 2 trials each
    for t in range(t0, t0 + 12):
        ro = o.trial(t)
        assert rg["trial"] == t and rg["move"] == ro["move"] and rg["flags"] & 0x3 == ro["flags"]
        if not ro["flags"]:
            for key in ("dH", "W_prot", "E_switch", "H0"):
                assert rel_close(rg[key], ro[key], 1e-6), (t, key, rg[key], ro[key])
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
        rg = g.trial()
    g.close()


def test_fp32_trials_lockstep():
    """Ten 200-step FP32 trials of a 2,000-ion box at the library's default
    lane count, each from the GPU's state against the FP64 oracle, within the
    FP32 bound |beta d(dH)| <= 1e-6 (N + |beta dH|) on dH and W_prot, with
    identical decisions outside it (the same check as tests/test_gpu_fp32.py
    makes at 4 lanes)."""
    from test_gpu_fp32 import compare_lockstep, lockstep
    say("case trials lj2000 fp32 lockstep, default lanes")
    w = W.lj_electrolyte(2000, 0.3, 21, n_steps=200, precision="fp32")
    w.params.update(beta_mu=6.0)
    g = h4d.System.from_workload(w)
    pairs = lockstep(g, w.params, (0,) * 10)
    compare_lockstep(pairs, 1.0, "lj2000/default lanes")
    g.close()


def ideal_closed_form(y, nmax=60):
    n = np.arange(nmax)
    logp = 2 * n * math.log(y) - 2 * np.array([math.lgamma(k + 1) for k in n])
    p = np.exp(logp - logp.max())
    return p / p.sum()


def test_ideal_reservoir_on_gpu():
    say("case ideal reservoir y=3")
    y, L = 3.0, 5.0
    w = W.ideal_gas(L=L, beta_mu=2 * math.log(y / L ** 3), n_steps=1)
    w.params.update(capacity=256)
    g = h4d.System.from_workload(w)
    recs = g.trials(20000, as_array=True)
    ns = np.array([recs[q].n_salt_after for q in range(20000)])[500:]
    emp = np.bincount(ns, minlength=60)[:60] / len(ns)
    tv = 0.5 * np.abs(emp - ideal_closed_form(y)).sum()
    say(f"   total variation {tv:.4f}, <N> {ns.mean():.3f}")
    assert tv < 0.03
    g.close()


def test_deletion_from_an_empty_box_is_a_rejected_attempt():
    say("case empty deletion")
    w = W.ideal_gas(L=6.0, beta_mu=0.0, n_steps=3)
    g = h4d.System.from_workload(w)
    r = g.trial(h4d.MOVE_DELETE)
    assert r["flags"] & h4d.FLAG_EMPTY and r["accepted"] == 0 and r["n_salt_after"] == 0
    g.close()


def test_trials_are_bitwise_deterministic():
    say("case determinism lj1000 fp32")
    w = W.lj_electrolyte(1000, 0.3, 31, n_steps=50, precision="fp32")
    w.params.update(beta_mu=8.0)
    a = h4d.System.from_workload(w)
    b = h4d.System.from_workload(w)
    ra, rb = a.trials(8), b.trials(8)
    for x, y in zip(ra, rb):
        assert x == y
    assert np.array_equal(a.state()["x"], b.state()["x"])
    a.close(); b.close()


def test_full_size_trials_32k_fp32():
    """The benchmark configuration at full size: the oracle recomputes each
    trial's starting Hamiltonian (FP64 energy of 32,000 ions plus the
    Maxwell-Boltzmann kinetic energy drawn for that trial) and the switch-on
    energy of an insertion; a rejected trial restores the state bitwise."""
    say("case trials lj32k fp32 (benchmark configuration, 4 trials)")
    w = W.config_lj_32k()
    g = h4d.System.from_workload(w)
    for t in range(4):
        st = g.state()
        o = O.OracleSystem(w.params, st["x"], st["type"], st["mol"], st["tag"], st["nsalt"],
                           cap=st["n"] + 8)
        ref = o.trial_begin(t)
        r = g.trial()
        say(f"   trial {t}: move {r['move']:+d} dH {r['dH']:.4f} shadow "
            f"{r['dH'] - r['E_switch'] - r['W_prot']:.4f} accepted {r['accepted']}")
        assert r["move"] == ref["move"] and r["n_steps"] == 200
        assert r["tag_c"] == ref["tag_c"] and r["tag_a"] == ref["tag_a"]
        assert r["H0"] == pytest.approx(ref["H0"], rel=1e-11)
        if r["move"] > 0:
            assert r["E_switch"] == pytest.approx(ref["E_switch"], rel=1e-9, abs=1e-9)
        assert math.isfinite(r["dH"]) and math.isfinite(r["W_prot"])
        after = g.state()
        if not r["accepted"]:
            assert np.array_equal(after["x"], st["x"]) and np.array_equal(after["tag"], st["tag"])
        assert after["n"] == 2 * after["nsalt"]
    g.close()


@pytest.mark.parametrize("schedule,n", [(1, 2.0), (2, 3.0)])
def test_variable_schedule_trials_match_oracle(schedule, n):
    say(f"case trials lj500 fp64, altitude schedule {schedule} (n = {n}), 20 trials")
    w = W.config_lj_500()
    w.params.update(beta_mu=6.0, schedule=schedule, schedule_n=n)
    g = h4d.System.from_workload(w)
    o = O.OracleSystem.from_workload(w, cap=w.n + 200)
    for t in range(20):
        rg, ro = g.trial(), o.trial(t)
        assert rg["move"] == ro["move"] and rg["flags"] & 0x3 == ro["flags"]
        if not ro["flags"]:
            for key in ("dH", "W_prot", "E_switch", "H0", "H1"):
                assert rel_close(rg[key], ro[key], 1e-6), (t, key, rg[key], ro[key])
        assert rg["accepted"] == ro["accepted"], (t, rg, ro)
    g.close()
