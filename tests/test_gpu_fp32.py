"""GPU parity of the FP32 pair pass at the launch shapes the benchmark times.

The FP32 mode computes pair forces in FP32 from 32-bit fixed-point
coordinates; positions, velocities, energies, work and the Metropolis ratio
stay FP64.  Its trajectories therefore leave the FP64 oracle's by rounding,
and the comparison runs in lockstep: before every trial the oracle restarts
from the GPU's state, and both run the same trial index (the same move,
sites and Maxwell-Boltzmann momenta from the shared Philox stream).

Checked here, for every lanes-per-atom width of the list traversal (4, 8 and
16; the autotuner picks 4 for eight 32,000-ion replicas and for the 256-box
batch, 16 for water):
* forces from one state, element by element (1e-5 relative, pairs within
  1e-6 of the Lennard-Jones cutoff may count either way);
* lockstep trials at the full 32,000-ion and aqueous NaCl sizes, with the
  flight shortened so the oracle stays within a minute;
* lockstep FP32 trials of a small water box, and of every box of a batch;
* the FP32 work distribution against the FP64 oracle's (paired trials, and a
  two-sample Kolmogorov-Smirnov test on disjoint trials).

FP32 bound on the work.  The FP32 force error (about 1e-6 relative, from
FP32 arithmetic on coordinates quantized to L 2^-32) is not the gradient of
the FP64 energy, so the FP32 trajectory's H drifts from the FP64 one's by a
sum over atoms and steps; a violent overlap (large beta dH) adds its own
share.  Measured lockstep differences |beta (dH_gpu - dH_oracle)| lie
between 1e-8 and 4e-7 per atom of the box (32,000 ions, 50 steps: 7e-4;
aqueous NaCl, 30 steps: 8.5e-3; 300 waters with beta dH up to 9,100: 1.1e-3).
The bound taken is
    |beta (dH_gpu - dH_oracle)| <= 1e-6 (N_atoms + |beta dH|),
three to ten times the measured spread, and the same bound on the protocol
work.  Decisions must agree whenever |ln u - ln R| exceeds that bound;
closer trials are flagged near-ties (none occurred in these runs).  A fixed
near-tie margin of 1e-4 cannot hold at these sizes: the FP32 spread of
beta dH itself exceeds it.
"""
import math
import sys

import numpy as np
import pytest

import oracle_pool
from paper_2307_11447_amd import h4d
from paper_2307_11447_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP32 bound on beta |dH_gpu - dH_oracle| per atom of the box and per kT of |beta dH|
FP32_DH_PER_ATOM = 1e-6


def fp32_tol(n_atoms, beta_dH):
    return FP32_DH_PER_ATOM * (n_atoms + abs(beta_dH))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pick_flyers(w):
    c = int(np.where(w.type == w.params["cation_type"])[0][3])
    a = int(np.where(w.type == w.params["anion_type"])[0][5])
    return c, a


def compare_lockstep(pairs, beta, label):
    """pairs: (GPU record, oracle record) of the same trial from the same
    state.  Returns the worst |beta d(dH)| relative to the FP32 bound."""
    worst = 0.0
    ties = 0
    for rg, ro in pairs:
        assert rg["trial"] == ro["trial"] and rg["move"] == ro["move"], (label, rg, ro)
        assert rg["flags"] & 0x3 == ro["flags"] & 0x3, (label, rg, ro)
        if ro["flags"] & 0x3:
            continue
        assert rg["tag_c"] == ro["tag_c"] and rg["tag_a"] == ro["tag_a"]
        assert rg["n_steps"] == ro["n_steps"]
        # the start state and its momenta are shared: FP64 energies agree
        assert rg["H0"] == pytest.approx(ro["H0"], rel=1e-11, abs=1e-9), (label, rg["trial"])
        if ro["move"] > 0:
            assert rg["E_switch"] == pytest.approx(ro["E_switch"], rel=1e-9, abs=1e-9)
        d = beta * abs(rg["dH"] - ro["dH"])
        dw = beta * abs(rg["W_prot"] - ro["W_prot"])
        tol_kt = fp32_tol(ro["n_atoms"] if "n_atoms" in ro else rg["n_atoms"], beta * ro["dH"])
        worst = max(worst, d / tol_kt)
        say(f"   {label} trial {rg['trial']}: move {ro['move']:+d} beta dH {beta * ro['dH']:.5f} "
            f"|beta d(dH)| {d:.2e} |beta d(W_prot)| {dw:.2e} bound {tol_kt:.2e} "
            f"margin {abs(ro['ln_u'] - ro['ln_ratio']):.2e}")
        assert d <= tol_kt, (label, rg["trial"], d)
        assert dw <= tol_kt, (label, rg["trial"], dw)
        if abs(ro["ln_u"] - ro["ln_ratio"]) > tol_kt:
            assert rg["accepted"] == ro["accepted"], (label, rg, ro)
        else:
            ties += 1
    say(f"   {label}: worst |beta d(dH)| at {worst:.3f} of the bound over {len(pairs)} trials ({ties} near-ties)")
    return worst


def lockstep(g, params, moves, n_mol=0, use_cells=True):
    """Run the GPU trials one by one, snapshotting the state before each, then
    the oracle's trials from those snapshots (in parallel)."""
    jobs, recs = [], []
    for mv in moves:
        st = g.state()
        r = g.trial(mv)
        recs.append(r)
        jobs.append(oracle_pool.job(params, st, r["trial"], mv, n_mol=n_mol, use_cells=use_cells))
    return list(zip(recs, oracle_pool.run(jobs)))


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_forces_32k_fp32_every_lane_width(lanes):
    from test_gpu_parity import compare_forces, cutoff_edge_terms, oracle_forces
    say(f"case forces n=32000 fp32, {lanes} lanes per atom")
    w = W.config_lj_32k()
    w.params.update(kappa_sr=0.5, lanes_per_atom=lanes)
    flyers = pick_flyers(w)
    g = h4d.System.from_workload(w)
    assert g.timing()["lanes"] == lanes
    Fg, eg = g.forces_at(flyers, 0.8)
    er, Fr = oracle_forces(w, flyers, 0.8)
    mask = np.ones(w.n, bool)
    mask[list(flyers)] = False
    compare_forces(Fg, Fr, mask, 1e-5, 1e-5, cutoff_edge_terms(w, flyers, 0.8))
    assert eg["U"] == pytest.approx(er.U, rel=1e-12)
    g.close()


@pytest.mark.parametrize("lanes", [4, 8])
def test_fp32_lockstep_lj32k_full_size(lanes):
    """The benchmark's 32,000-ion box at its density, skin and lane width,
    with the flight cut to 50 steps: two insertions and two deletions."""
    say(f"case fp32 lockstep lj32k full size, {lanes} lanes, N_f = 50")
    w = W.config_lj_32k()
    w.params.update(n_steps=50, lanes_per_atom=lanes, beta_mu=-7.6, capacity=w.n + 1024)
    g = h4d.System.from_workload(w)
    pairs = lockstep(g, w.params, (1, -1, 1, -1))
    compare_lockstep(pairs, 1.0, f"lj32k/L{lanes}")
    g.close()


def test_fp32_lockstep_lj2000_full_flight():
    """A 2,000-ion box with the benchmark's full 200-step flight."""
    say("case fp32 lockstep lj2000, N_f = 200, 4 lanes")
    w = W.lj_electrolyte(2000, 0.3, 21, n_steps=200, precision="fp32")
    w.params.update(beta_mu=6.0, lanes_per_atom=4)
    g = h4d.System.from_workload(w)
    pairs = lockstep(g, w.params, (0,) * 10)
    compare_lockstep(pairs, 1.0, "lj2000/L4")
    g.close()


@pytest.mark.parametrize("lanes,loads", [(4, -1), (16, -1), (8, 1)])
def test_fp32_lockstep_water_full_size(lanes, loads):
    """The aqueous NaCl box (8,000 rigid waters + 150 pairs, 62 A) with the
    flight cut to 30 steps of 1 fs: one insertion and one deletion.  The
    third case runs the instantiation the bench times on this machine's eight
    replicas: 8 lanes per atom with non-temporal list loads."""
    say(f"case fp32 lockstep aqueous NaCl full size, {lanes} lanes, list loads {loads}, N_f = 30")
    w = W.config_water_nacl()
    w.params.update(n_steps=30, lanes_per_atom=lanes, beta_mu=-120.0)
    beta = 1.0 / w.params["kT"]
    g = h4d.System.from_workload(w)
    g.set_list_loads(loads)
    if loads >= 0:
        assert g.timing()["nt_lists"] == loads
    pairs = lockstep(g, w.params, (1, -1), n_mol=w.n_mol)
    compare_lockstep(pairs, beta, f"water/L{lanes}/loads{loads}")
    g.close()


def test_list_load_kinds_give_identical_trials():
    """The pair pass with cached and with non-temporal list-index loads gives
    the same records and states, bitwise (an FP32 batch of small boxes,
    three rounds from the same start)."""
    from test_gpu_batch import small_boxes
    say("case list-load kinds, fp32 batch, 3 rounds each")
    out = []
    for mode in (0, 1):
        ws = small_boxes("fp32", 30, 60, seed=2202)
        bat = h4d.Batch.from_workloads(ws)
        bat.set_list_loads(mode)
        assert bat.timing()["nt_lists"] == mode
        recs = bat.run(3)
        out.append((recs, [bat.box_state(b) for b in range(len(ws))]))
        bat.close()
    (r0, s0), (r1, s1) = out
    for b in range(len(r0)):
        for q in range(3):
            for k in ("move", "accepted", "trial", "n_steps", "dH", "W_prot", "E_switch"):
                assert r0[b][q][k] == r1[b][q][k], (b, q, k, r0[b][q][k], r1[b][q][k])
        assert np.array_equal(s0[b]["x"], s1[b]["x"]), b


@pytest.mark.parametrize("lanes", [4, 16])
def test_fp32_water_lockstep_small(lanes):
    """FP32 water trajectories against the oracle (300 waters + 10 pairs,
    20-step flights): energies, work, decisions and rigid geometry."""
    from test_gpu_water import bond_error, box
    say(f"case fp32 water lockstep, 300 waters, {lanes} lanes")
    w = box(300, 10, 21.0, 7, 78, precision="fp32", n_steps=20, beta_mu=20.0, lanes_per_atom=lanes)
    beta = 1.0 / w.params["kT"]
    g = h4d.System.from_workload(w)
    pairs = lockstep(g, w.params, (0,) * 12, n_mol=300, use_cells=False)
    compare_lockstep(pairs, beta, f"water300/L{lanes}")
    assert sum(rg["accepted"] for rg, _ in pairs) >= 1
    assert bond_error(g.state()["x"], w, 300) < 1e-9
    g.close()


@pytest.mark.parametrize("lanes", [4, 8])
def test_fp32_batch_lockstep_per_box(lanes):
    """Every box of an FP32 batch, one round at a time, against the oracle
    restarted from that box's state (each box its own stream and N_f)."""
    from test_gpu_batch import small_boxes
    say(f"case fp32 batch lockstep per box, {lanes} lanes")
    ws = small_boxes("fp32", 30, 60, seed=2201)
    for w in ws:
        w.params.update(lanes_per_atom=lanes)
    bat = h4d.Batch.from_workloads(ws)
    assert bat.timing()["lanes"] == lanes
    pairs = {b: [] for b in range(len(ws))}
    for rnd in range(4):
        states = [bat.box_state(b) for b in range(len(ws))]
        recs = bat.run(1)
        jobs = [oracle_pool.job(ws[b].params, states[b], recs[b][0]["trial"]) for b in range(len(ws))]
        for b, ro in enumerate(oracle_pool.run(jobs)):
            pairs[b].append((recs[b][0], ro))
    for b in range(len(ws)):
        compare_lockstep(pairs[b], 1.0, f"batch box {b}/L{lanes}")
    bat.close()


def test_fp32_full_size_batch_lockstep_sampled_boxes():
    """The full 256-box batch (2.2 M ions, N in [1000, 16000], density
    0.1-0.4, N_f ~ U{100..400}) at the 4 lanes per atom the bench tunes to,
    with the non-temporal list loads its size selects (the instantiation the
    bench times): one round, and for a sample of boxes (the smallest, the
    largest and three others) the oracle's whole trial from that box's start
    state within the FP32 bound, with the same move, sites, N_f and
    decision."""
    say("case fp32 full-size batch (256 boxes), one round, 5 boxes through the oracle")
    ws = W.config_batched()
    for w in ws:
        w.params.update(lanes_per_atom=4)
    sizes = [w.n for w in ws]
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0, 77, 254})
    bat = h4d.Batch.from_workloads(ws)
    tm = bat.timing()
    assert tm["lanes"] == 4 and tm["nt_lists"] == 1
    states = {b: bat.box_state(b) for b in sample}
    recs = bat.run(1)
    jobs = [oracle_pool.job(ws[b].params, states[b], recs[b][0]["trial"]) for b in sample]
    for b, ro in zip(sample, oracle_pool.run(jobs)):
        say(f"   box {b}: {sizes[b]} ions, N_f {recs[b][0]['n_steps']}")
        compare_lockstep([(recs[b][0], ro)], 1.0, f"full batch box {b}")
    assert all(100 <= r[0]["n_steps"] <= 400 for r in recs)
    bat.close()


def test_fp32_work_distribution_against_fp64():
    """Forced insertions and deletions on one fixed state (beta mu = -+1000:
    never accepted, so the state does not change).  Paired: GPU FP32 and
    oracle FP64 trials with the same indices agree within the FP32 bound.
    Unpaired: the FP32 works of trials 0..119 and the FP64 works of trials
    120..239 are samples of one distribution (two-sample Kolmogorov-Smirnov,
    p > 1e-3)."""
    from scipy import stats
    say("case fp32 vs fp64 work distributions, 1000 ions, N_f = 100, 4 lanes")
    w = W.lj_electrolyte(1000, 0.3, 1201, n_steps=100, precision="fp32")
    w.params.update(lanes_per_atom=4)
    g = h4d.System.from_workload(w)
    st = g.state()
    n = 60
    gpu = {}
    for move, bm in ((1, -1.0e3), (-1, 1.0e3)):
        g.set_beta_mu(bm)
        for r in g.trials(n, move):
            gpu[r["trial"]] = r
    assert np.array_equal(g.state()["x"], st["x"])    # no move was accepted
    g.close()
    ins_t, del_t = list(range(n)), list(range(n, 2 * n))
    jobs = []
    for ts, move, bm in ((ins_t, 1, -1.0e3), (del_t, -1, 1.0e3)):
        for t in ts:                     # paired: the same trial indices
            jobs.append(oracle_pool.job(dict(w.params, beta_mu=bm), st, t, move))
        for t in ts:                     # unpaired: later indices
            jobs.append(oracle_pool.job(dict(w.params, beta_mu=bm), st, t + 2 * n, move))
    orc = oracle_pool.run(jobs)
    o_ins, o_ins_late, o_del, o_del_late = orc[:n], orc[n:2 * n], orc[2 * n:3 * n], orc[3 * n:]
    worst = 0.0
    for ro in o_ins + o_del:
        rg = gpu[ro["trial"]]
        assert rg["move"] == ro["move"] and rg["tag_c"] == ro["tag_c"] and rg["tag_a"] == ro["tag_a"]
        if not ro["flags"]:
            worst = max(worst, abs(rg["dH"] - ro["dH"]) / fp32_tol(w.n, ro["dH"]))
    say(f"   paired: worst |beta d(dH)| at {worst:.3f} of the FP32 bound")
    assert worst <= 1.0
    for name, g_recs, o_recs in (("insertion", [gpu[t] for t in ins_t], o_ins_late),
                                 ("deletion", [gpu[t] for t in del_t], o_del_late)):
        a = np.array([r["dM"] for r in g_recs if not r["flags"] & 0x3])
        b = np.array([r["dM"] for r in o_recs if not r["flags"] & 0x3])
        res = stats.ks_2samp(a, b)
        say(f"   {name}: FP32 <dM> {a.mean():.3f} (sd {a.std():.3f}), FP64 <dM> {b.mean():.3f} "
            f"(sd {b.std():.3f}), KS D {res.statistic:.3f} p {res.pvalue:.3f}")
        assert res.pvalue > 1e-3
