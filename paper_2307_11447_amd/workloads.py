"""Seeded synthetic workloads (inputs only, no arithmetic of the method).

These generators produce the model parameters and the starting
configuration of each workload.  Both the GPU library (through its Python
binding) and the CPU oracle (through the tests) consume them, so they
contain no part of the pair potentials, the integrator, the work or the
acceptance rule: only positions, types, tags and parameter values.

Workloads (all cubic periodic boxes):

* ``lj_electrolyte``: the paper's Lennard-Jones ions (Sec. II D 1):
  sigma = epsilon = m = 1, charges +-1, LJ truncated and shifted at
  2.5 sigma, reduced Coulomb with a Bjerrum length of 3 sigma
  (coulomb_k = 3 at kT = 1), damped shifted force with alpha = 0.3 and a
  4 sigma cutoff.  Start: a jittered simple-cubic lattice (nearest
  distance >= 0.9 sigma) with random site occupation and random charges.
* ``water_nacl``: SPC/E water plus Joung-Cheatham-like Na+/Cl- with
  Lorentz-Berthelot mixing (Sec. II D 2), real units (kcal/mol, A, fs,
  amu, e), 298 K, rigid waters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Real-unit constants (kcal/mol, Angstrom, fs, amu, elementary charge).
COULOMB_K_REAL = 332.0637          # kcal A / (mol e^2)
KB_REAL = 0.0019872043             # kcal / (mol K)
ACCEL_REAL = 4.184e-4              # A/fs^2 per (kcal/mol/A)/amu


@dataclass
class Workload:
    """Parameters (a flat dict of physical values) and a starting state."""
    name: str
    params: dict
    x: np.ndarray          # (n, 3) float64, wrapped into [0, L)
    type: np.ndarray       # (n,) int32
    mol: np.ndarray        # (n,) int32, -1 for ions
    tag: np.ndarray        # (n,) int64
    nsalt: int
    n_mol: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _base_lj_params(L: float) -> dict:
    return dict(
        n_types=2, cation_type=0, anion_type=1,
        mass=[1.0, 1.0], charge=[1.0, -1.0], sigma=[1.0, 1.0], eps=[1.0, 1.0],
        box=[L, L, L], kT=1.0, dt=0.005, w_max=2.5, kappa_sr=0.0,
        rc_lj=2.5, rc_coul=4.0, alpha=0.3, coulomb_k=3.0,
        beta_mu=0.0, lambda_s=1.0, n_steps=100, n_steps_min=0, n_steps_max=0,
        water=0, d_oh=0.0, d_hh=0.0, accel=1.0,
        seed=1000, stream=0, skin=0.5, precision="fp64",
    )


def jittered_lattice(n: int, L: float, min_dist: float, rng: np.random.Generator) -> np.ndarray:
    """n points in [0, L)^3 on randomly chosen sites of a simple-cubic
    lattice, each displaced uniformly so that no two are closer than
    min_dist (periodic)."""
    m = int(math.ceil(n ** (1.0 / 3.0)))
    while m ** 3 < n:
        m += 1
    a = L / m
    if a <= min_dist:
        raise ValueError(f"density too high for a {min_dist} spacing")
    jit = 0.5 * (a - min_dist)
    sites = rng.choice(m ** 3, size=n, replace=False)
    ijk = np.stack([sites % m, (sites // m) % m, sites // (m * m)], axis=1).astype(np.float64)
    x = (ijk + 0.5) * a + rng.uniform(-jit, jit, size=(n, 3))
    return np.mod(x, L)


def lj_electrolyte(n_atoms: int, density: float, seed: int, *, n_steps: int = 100,
                   precision: str = "fp64", name: str = "lj") -> Workload:
    if n_atoms % 2:
        raise ValueError("n_atoms must be even (charge neutral)")
    L = (n_atoms / density) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    x = jittered_lattice(n_atoms, L, 0.9, rng)
    types = np.zeros(n_atoms, dtype=np.int32)
    types[rng.permutation(n_atoms)[: n_atoms // 2]] = 1
    p = _base_lj_params(L)
    p.update(seed=seed, n_steps=n_steps, precision=precision)
    # keep every species' atoms in ascending tag order with tags 0..n-1
    return Workload(name=name, params=p, x=x, type=types,
                    mol=np.full(n_atoms, -1, np.int32),
                    tag=np.arange(n_atoms, dtype=np.int64), nsalt=n_atoms // 2)


# ---------------------------------------------------------------------------
# The five benchmark configurations (seed 1000 + c).
# ---------------------------------------------------------------------------

def config_lj_500() -> Workload:
    """500 LJ ions at density 0.3, 100 steps of dt 0.005, w from 2.5 to 0, FP64."""
    return lj_electrolyte(500, 0.3, 1001, n_steps=100, precision="fp64", name="lj500_fp64")


def config_lj_32k() -> Workload:
    """32,000 LJ ions at density 0.3, 200 NEMD steps, FP32 forces / FP64 work."""
    w = lj_electrolyte(32000, 0.3, 1002, n_steps=200, precision="fp32", name="lj32k_fp32")
    return w


def config_batched(n_boxes: int = 256, seed: int = 1003):
    """Replica boxes: N_b even in [1000, 16000], density U[0.1, 0.4],
    N_f ~ U{100..400} per trial (drawn by the method's own generator)."""
    rng = np.random.default_rng(seed)
    boxes = []
    for b in range(n_boxes):
        n = 1000 + 2 * int(rng.integers(0, 7501))
        rho = float(rng.uniform(0.1, 0.4))
        w = lj_electrolyte(n, rho, seed * 1000 + b, n_steps=0, precision="fp32",
                           name=f"box{b}")
        w.params.update(n_steps=0, n_steps_min=100, n_steps_max=400, stream=b, seed=seed)
        boxes.append(w)
    return boxes


def _water_params(L: float) -> dict:
    kT = KB_REAL * 298.0
    return dict(
        # types: 0 O, 1 H, 2 Na, 3 Cl
        n_types=4, cation_type=2, anion_type=3,
        mass=[15.9994, 1.008, 22.98977, 35.453],
        charge=[-0.8476, 0.4238, 1.0, -1.0],
        sigma=[3.166, 0.0, 2.16, 4.83],
        eps=[0.1553, 0.0, 0.35, 0.0128],
        box=[L, L, L], kT=kT, dt=1.0, w_max=3.0, kappa_sr=1.0,
        rc_lj=10.0, rc_coul=10.0, alpha=0.25, coulomb_k=COULOMB_K_REAL,
        beta_mu=0.0, lambda_s=1.0, n_steps=500, n_steps_min=0, n_steps_max=0,
        water=1, d_oh=1.0, d_hh=2.0 * math.sin(math.radians(109.47) / 2.0),
        accel=ACCEL_REAL, seed=1004, stream=0, skin=1.0, precision="fp32",
    )


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def water_nacl(n_water: int = 8000, n_pairs: int = 150, L: float = 62.0, m: int = 21,
               seed: int = 1004, name: str = "nacl_water", tries: int = 24) -> Workload:
    """Rigid SPC/E waters and Na+/Cl- on randomly chosen sites of an m^3
    lattice.  Each water's orientation is the best of `tries` random
    rotations: the one whose hydrogens stay farthest from the neighbouring
    occupied sites (hydrogens carry no Lennard-Jones core, so a hydrogen
    placed against a neighbour would collapse onto it).  Atom layout: waters
    first (O, H, H of molecule k at 3k..3k+2), then the ions; tags ascending."""
    rng = np.random.default_rng(seed)
    p = _water_params(L)
    p["seed"] = seed
    a = L / m
    if n_water + 2 * n_pairs > m ** 3:
        raise ValueError("lattice too small")
    sites = rng.choice(m ** 3, size=n_water + 2 * n_pairs, replace=False)
    ijk = np.stack([sites % m, (sites // m) % m, sites // (m * m)], axis=1)
    centers = (ijk.astype(np.float64) + 0.5) * a
    occupied = np.full((m, m, m), -1, dtype=np.int64)
    occupied[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = np.arange(len(sites))
    shell = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
                      if (dx, dy, dz) != (0, 0, 0)])
    half = 0.5 * p["d_hh"]
    h_off = math.sqrt(p["d_oh"] ** 2 - half ** 2)
    body = np.array([[0.0, 0.0, 0.0], [half, h_off, 0.0], [-half, h_off, 0.0]])
    xs, ts, ms = [], [], []
    for k in range(n_water):
        nb = (ijk[k] + shell) % m
        occ = occupied[nb[:, 0], nb[:, 1], nb[:, 2]] >= 0
        rel = shell[occ].astype(np.float64) * a          # neighbouring sites relative to this one
        best, best_d = None, -1.0
        for _ in range(tries):
            R = _random_rotation(rng)
            hpos = body[1:] @ R.T
            d = np.min(np.linalg.norm(hpos[:, None, :] - rel[None, :, :], axis=2)) if len(rel) else 9.9
            if d > best_d:
                best, best_d = R, d
        xs.append(centers[k] + body @ best.T)
        ts += [0, 1, 1]
        ms += [k, k, k]
    ion_types = np.array([2] * n_pairs + [3] * n_pairs, dtype=np.int32)
    rng.shuffle(ion_types)
    x = np.concatenate([np.concatenate(xs, axis=0), centers[n_water:]], axis=0) if n_water else centers
    t = np.concatenate([np.array(ts, np.int32), ion_types])
    mol = np.concatenate([np.array(ms, np.int32), np.full(2 * n_pairs, -1, np.int32)])
    n = x.shape[0]
    return Workload(name=name, params=p, x=np.mod(x, L), type=t, mol=mol,
                    tag=np.arange(n, dtype=np.int64), nsalt=n_pairs, n_mol=n_water)


def config_water_nacl() -> Workload:
    """8,000 SPC/E waters + 150 NaCl pairs in a 62 A box, 500-step NEMD, dt 1 fs."""
    return water_nacl()


def small_lj(n_atoms: int = 64, density: float = 0.3, seed: int = 7, n_steps: int = 20,
             precision: str = "fp64") -> Workload:
    """A small LJ-ion box for parity tests."""
    return lj_electrolyte(n_atoms, density, seed, n_steps=n_steps, precision=precision,
                          name=f"lj{n_atoms}")


def ideal_gas(L: float, beta_mu: float, n_steps: int = 2, seed: int = 11) -> Workload:
    """Ions with no interactions at all (epsilon = 0, q = 0): the exact
    stationary distribution of N is known in closed form."""
    p = _base_lj_params(L)
    p.update(charge=[0.0, 0.0], eps=[0.0, 0.0], beta_mu=beta_mu, n_steps=n_steps, seed=seed,
             rc_lj=min(2.5, 0.45 * L), rc_coul=min(4.0, 0.45 * L), w_max=min(2.5, 0.45 * L))
    return Workload(name="ideal", params=p, x=np.zeros((0, 3)), type=np.zeros(0, np.int32),
                    mol=np.zeros(0, np.int32), tag=np.zeros(0, np.int64), nsalt=0)
