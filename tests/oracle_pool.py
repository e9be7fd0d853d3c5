"""Oracle trials in parallel CPU processes (test infrastructure).

A lockstep comparison restarts the oracle from the GPU's state before every
trial, so the oracle's trials are independent jobs: each rebuilds an
OracleSystem from a state snapshot and runs one trial.  The worker processes
are spawned (no inherited GPU context), import only numpy and the oracle, and
never touch the GPU.
"""
import multiprocessing as mp
import os


def _job(args):
    from oracle import oracle as O
    params, x, type_, mol, tag, nsalt, n_mol, t, move, use_cells = args
    o = O.OracleSystem(params, x, type_, mol, tag, nsalt, n_mol=n_mol, cap=len(type_) + 8, use_cells=use_cells)
    return o.trial(t, move)


def job(params, st, t, move=0, n_mol=0, use_cells=True):
    """One oracle trial t (forced move, or 0) from the state snapshot st
    (a dict with x, type, mol, tag, nsalt as returned by state())."""
    return (dict(params), st["x"], st["type"], st["mol"], st["tag"], int(st["nsalt"]), n_mol, int(t), int(move),
            use_cells)


def run(jobs, procs=None):
    """Records of the jobs, in order.  At most 12 processes (the host of one
    GPU gives a process 16 threads)."""
    if not jobs:
        return []
    procs = procs or max(1, min(len(jobs), 12, os.cpu_count() or 1))
    if procs == 1:
        return [_job(j) for j in jobs]
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.map(_job, jobs, chunksize=1)
