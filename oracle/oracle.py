"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` built from
``h4d_oracle.c`` by ``oracle/build.py`` and shares nothing with the GPU
library except the seeded workload generators that feed both.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")
MAXT = 8

MODE_NEMD, MODE_EXCL, MODE_FLY = 0, 1, 2
FLAG_EMPTY, FLAG_NONFINITE, FLAG_INSTANT = 1, 2, 16


class Params(C.Structure):
    _fields_ = [
        ("n_types", C.c_int32), ("cation_type", C.c_int32), ("anion_type", C.c_int32),
        ("n_steps", C.c_int32), ("n_steps_min", C.c_int32), ("n_steps_max", C.c_int32),
        ("water", C.c_int32), ("use_cells", C.c_int32),
        ("mass", C.c_double * MAXT), ("charge", C.c_double * MAXT),
        ("sigma", C.c_double * MAXT), ("eps", C.c_double * MAXT),
        ("box", C.c_double * 3),
        ("kT", C.c_double), ("dt", C.c_double), ("w_max", C.c_double), ("kappa_sr", C.c_double),
        ("rc_lj", C.c_double), ("rc_coul", C.c_double), ("alpha", C.c_double), ("ke", C.c_double),
        ("beta_mu", C.c_double), ("lambda_s", C.c_double),
        ("d_oh", C.c_double), ("d_hh", C.c_double), ("accel", C.c_double),
        ("seed", C.c_uint64), ("stream", C.c_uint64),
        ("bias_xb", C.c_double), ("bias_alpha", C.c_double),
        ("schedule", C.c_int32), ("schedule_n", C.c_double),
        ("momenta", C.c_int32), ("md_refresh", C.c_double),
        ("w_max_ratio", C.c_double), ("v_ex_edge", C.c_double),
    ]


class State(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("cap", C.c_int32), ("nsalt", C.c_int32), ("n_mol", C.c_int32),
        ("next_tag", C.c_int64),
        ("x", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
        ("type", C.POINTER(C.c_int32)), ("mol", C.POINTER(C.c_int32)),
        ("tag", C.POINTER(C.c_int64)), ("flying", C.POINTER(C.c_int32)),
    ]


class TrialRec(C.Structure):
    _fields_ = [
        ("move", C.c_int32), ("accepted", C.c_int32), ("n_salt_before", C.c_int32),
        ("n_salt_after", C.c_int32), ("n_steps", C.c_int32), ("flags", C.c_int32),
        ("trial", C.c_int64), ("tag_c", C.c_int64), ("tag_a", C.c_int64),
        ("dH", C.c_double), ("dU", C.c_double), ("dK", C.c_double), ("W_prot", C.c_double),
        ("E_switch", C.c_double), ("dM", C.c_double), ("ln_ratio", C.c_double),
        ("ln_u", C.c_double), ("ln_proposal", C.c_double), ("H0", C.c_double), ("H1", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


LOGIT_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double))


class Proposal(C.Structure):
    _fields_ = [("k", C.c_int32), ("fn", LOGIT_FN), ("ctx", C.c_void_p), ("cap", C.c_double),
                ("scale", C.c_double)]


class Energy(C.Structure):
    _fields_ = [("U", C.c_double), ("U_lj", C.c_double), ("U_c", C.c_double),
                ("virial", C.c_double), ("dUdw", C.c_double)]


_lib = None


def use_timing_build() -> str:
    """Switch this process to the OpenMP build of the same source (thread
    count from OMP_NUM_THREADS): for the benchmark's CPU-baseline timing
    only; every parity check uses the single-threaded build.  Call before
    anything else loads the oracle."""
    global _lib
    if _lib is not None and getattr(_lib, "_path", None) != LIB_OMP_PATH:
        raise RuntimeError("the oracle is already loaded single-threaded")
    _lib = None
    return lib(LIB_OMP_PATH)._path


def lib(path=None):
    global _lib
    if _lib is None:
        path = path or LIB_PATH
        if not os.path.exists(path):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(path)
        L._path = path
        P, S = C.POINTER(Params), C.POINTER(State)
        L.or_philox4x64.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.or_u01.argtypes = [C.c_uint64]
        L.or_u01.restype = C.c_double
        L.or_pair.argtypes = [P, C.c_int, C.c_int, C.c_double, C.c_double] + [C.POINTER(C.c_double)] * 4
        L.or_compute.argtypes = [P, S, C.c_double, C.c_int, C.POINTER(C.c_double), C.POINTER(Energy)]
        L.or_mb_velocities.argtypes = [P, S, C.c_uint64]
        L.or_constrain_positions.argtypes = [P, S, C.POINTER(C.c_double)]
        L.or_constrain_velocities.argtypes = [P, S]
        L.or_kinetic.argtypes = [P, S]
        L.or_kinetic.restype = C.c_double
        L.or_altitude.argtypes = [P, C.c_int, C.c_int, C.c_int]
        L.or_altitude.restype = C.c_double
        L.or_nemd.argtypes = [P, S, C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.or_trial.argtypes = [P, S, C.c_uint64, C.c_int, C.POINTER(TrialRec)]
        L.or_trial_begin.argtypes = [P, S, C.c_uint64, C.c_int, C.POINTER(TrialRec),
                                     C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.or_mtm_log_factor.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                                        C.POINTER(C.c_double)]
        L.or_site_features.argtypes = [P, S, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_bias_b.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_bias_b.restype = C.c_double
        L.or_bias_B.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_bias_B.restype = C.c_double
        L.or_bias_offset.argtypes = [P, C.c_uint64, C.c_int]
        L.or_bias_offset.restype = C.c_double
        L.or_trial_learned.argtypes = [P, S, C.c_uint64, C.c_int, C.POINTER(Proposal), C.POINTER(TrialRec),
                                       C.POINTER(C.c_double)]
        L.or_init_velocities.argtypes = [P, S]
        L.or_md_phase.argtypes = [P, S, C.c_uint64, C.c_int, C.POINTER(TrialRec)]
        _lib = L
    return _lib


def make_params(d: dict, use_cells: bool = True) -> Params:
    p = Params()
    p.n_types = d["n_types"]
    p.cation_type, p.anion_type = d["cation_type"], d["anion_type"]
    p.n_steps = d["n_steps"]
    p.n_steps_min, p.n_steps_max = d.get("n_steps_min", 0), d.get("n_steps_max", 0)
    p.water = d.get("water", 0)
    p.use_cells = 1 if use_cells else 0
    for name in ("mass", "charge", "sigma", "eps"):
        arr = getattr(p, name)
        for i, v in enumerate(d[name]):
            arr[i] = v
    for i in range(3):
        p.box[i] = d["box"][i]
    for k in ("kT", "dt", "w_max", "kappa_sr", "rc_lj", "rc_coul", "alpha",
              "beta_mu", "lambda_s", "d_oh", "d_hh"):
        setattr(p, k, d[k])
    p.ke = d["coulomb_k"]
    p.accel = d.get("accel", 1.0)
    p.seed, p.stream = d["seed"], d.get("stream", 0)
    p.bias_xb, p.bias_alpha = d.get("bias_xb", 0.0), d.get("bias_alpha", 0.0)
    p.schedule, p.schedule_n = d.get("schedule", 0), d.get("schedule_n", 1.0)
    p.momenta, p.md_refresh = d.get("momenta", 0), d.get("md_refresh", 0.0)
    p.w_max_ratio = d.get("w_max_ratio", 0.0)
    p.v_ex_edge = d.get("v_ex_edge", 0.0)
    return p


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


class OracleSystem:
    """A configuration plus model parameters, advanced by the C oracle."""

    def __init__(self, params: dict, x, type_, mol, tag, nsalt: int, n_mol: int = 0,
                 cap: int | None = None, use_cells: bool = True):
        n = len(type_)
        cap = cap or (n + 64)
        self.pd = dict(params)
        self.p = make_params(params, use_cells)
        self.x = np.zeros((cap, 3)); self.x[:n] = x
        self.v = np.zeros((cap, 3))
        self.type = np.zeros(cap, np.int32); self.type[:n] = type_
        self.mol = np.full(cap, -1, np.int32); self.mol[:n] = mol
        self.tag = np.zeros(cap, np.int64); self.tag[:n] = tag
        self.flying = np.zeros(cap, np.int32)
        self.s = State()
        self.s.n, self.s.cap, self.s.nsalt, self.s.n_mol = n, cap, nsalt, n_mol
        self.s.next_tag = int(tag.max()) + 1 if n else 0
        self.s.x, self.s.v = _dp(self.x), _dp(self.v)
        self.s.type, self.s.mol = _ip(self.type), _ip(self.mol)
        self.s.tag, self.s.flying = _lp(self.tag), _ip(self.flying)
        if n:
            rc = lib().or_init_velocities(C.byref(self.p), C.byref(self.s))
            if rc:
                raise RuntimeError(f"or_init_velocities failed: {rc}")

    @classmethod
    def from_workload(cls, w, cap=None, use_cells=True):
        return cls(w.params, w.x, w.type, w.mol, w.tag, w.nsalt, w.n_mol, cap, use_cells)

    @property
    def n(self):
        return self.s.n

    @property
    def nsalt(self):
        return self.s.nsalt

    def compute(self, w: float = 0.0, mode: int = MODE_NEMD, forces: bool = True):
        F = np.zeros((self.n, 3)) if forces else None
        e = Energy()
        rc = lib().or_compute(C.byref(self.p), C.byref(self.s), w, mode,
                              _dp(F) if forces else None, C.byref(e))
        if rc:
            raise RuntimeError(f"or_compute failed: {rc}")
        return e, F

    def trial(self, t: int, force_move: int = 0) -> dict:
        rec = TrialRec()
        rc = lib().or_trial(C.byref(self.p), C.byref(self.s), t, force_move, C.byref(rec))
        if rc:
            raise RuntimeError(f"or_trial failed: {rc}")
        return rec.as_dict()

    def md_phase(self, phase: int, n_steps: int) -> dict:
        """Equilibrium phase `phase` (generalized hybrid MC, n_steps steps)."""
        rec = TrialRec()
        rc = lib().or_md_phase(C.byref(self.p), C.byref(self.s), phase, n_steps, C.byref(rec))
        if rc:
            raise RuntimeError(f"or_md_phase failed: {rc}")
        return rec.as_dict()

    def velocities(self):
        return self.v[: self.n].copy()

    def site_features(self, site) -> np.ndarray:
        """Features (64) of the pair site (cation xyz, anion xyz) on the
        current state without its flying atoms."""
        st = np.ascontiguousarray(site, dtype=np.float64).reshape(6)
        out = np.zeros(64)
        rc = lib().or_site_features(C.byref(self.p), C.byref(self.s), _dp(st), _dp(out))
        if rc:
            raise RuntimeError(f"or_site_features failed: {rc}")
        return out

    def trial_learned(self, t: int, k: int, logits=None, force_move: int = 0, cap: float = 10.0,
                      scale: float = 1.0):
        """Trial with the learned proposal.  logits(features n x 64) -> n
        logits, or None for equal weights; log weights are
        scale * min(logit, cap).  Returns (record, features of the inserted /
        removed site)."""
        prop = Proposal()
        prop.k = k
        prop.cap = cap
        prop.scale = scale
        keep = None
        if logits is not None:
            def cb(ctx, n, feat, out):
                try:
                    X = np.ctypeslib.as_array(feat, shape=(n, 64)).copy()
                    s = np.asarray(logits(X), dtype=np.float64).reshape(n)
                    for j in range(n):
                        out[j] = float(s[j])
                    return 0
                except Exception:
                    return -1
            keep = LOGIT_FN(cb)
            prop.fn = keep
        rec = TrialRec()
        feat = np.zeros(64)
        rc = lib().or_trial_learned(C.byref(self.p), C.byref(self.s), t, force_move, C.byref(prop),
                                    C.byref(rec), _dp(feat))
        if rc:
            raise RuntimeError(f"or_trial_learned failed: {rc}")
        del keep
        return rec.as_dict(), feat

    def trial_begin(self, t: int, force_move: int = 0) -> dict:
        """Proposal, momenta, H_start and (insertion) switch-on energy of
        trial t; leaves the flyers marked in this state."""
        rec = TrialRec()
        ic, ia, nf = C.c_int(), C.c_int(), C.c_int()
        rc = lib().or_trial_begin(C.byref(self.p), C.byref(self.s), t, force_move, C.byref(rec),
                                  C.byref(ic), C.byref(ia), C.byref(nf))
        if rc < 0:
            raise RuntimeError(f"or_trial_begin failed: {rc}")
        d = rec.as_dict()
        d.update(ic=ic.value, ia=ia.value, nf=nf.value, proceeds=rc)
        return d

    def mb(self, t: int):
        rc = lib().or_mb_velocities(C.byref(self.p), C.byref(self.s), t)
        if rc:
            raise RuntimeError(f"or_mb_velocities failed: {rc}")

    def kinetic(self) -> float:
        return lib().or_kinetic(C.byref(self.p), C.byref(self.s))

    def nemd(self, move: int, nf: int) -> float:
        W = C.c_double()
        rc = lib().or_nemd(C.byref(self.p), C.byref(self.s), move, nf, C.byref(W))
        if rc:
            raise RuntimeError(f"or_nemd failed: {rc}")
        return W.value

    def positions(self):
        return self.x[: self.n].copy()


def philox4x64(ctr, key):
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().or_philox4x64(c, k, o)
    return [int(v) for v in o]


def u01(bits: int) -> float:
    return lib().or_u01(bits)


def pair(params: dict, ti: int, tj: int, s: float, g: float = 1.0):
    p = make_params(params)
    out = [C.c_double() for _ in range(4)]
    lib().or_pair(C.byref(p), ti, tj, s * s, g, *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def mtm_log_factor(move: int, logw, sel: int) -> float:
    a = np.ascontiguousarray(logw, dtype=np.float64)
    out = C.c_double()
    rc = lib().or_mtm_log_factor(move, len(a), _dp(a), sel, C.byref(out))
    if rc:
        raise ValueError("bad arguments")
    return out.value


def bias_b(x: float, L: float, xb: float, alpha: float) -> float:
    """b_ins of Eq. (14) (bimodal bias of the anion offset along one edge)."""
    return lib().or_bias_b(x, L, xb, alpha)


def bias_B(params: dict, xa, xc) -> float:
    """B_ins of Eq. (12) for an anion at xa and a cation at xc."""
    p = make_params(params)
    a = np.ascontiguousarray(xa, dtype=np.float64)
    c = np.ascontiguousarray(xc, dtype=np.float64)
    return lib().or_bias_B(C.byref(p), _dp(a), _dp(c))


def bias_offset(params: dict, trial: int, d: int) -> float:
    """The anion offset of an insertion along edge d (a draw from Eq. 14)."""
    p = make_params(params)
    return lib().or_bias_offset(C.byref(p), trial, d)
