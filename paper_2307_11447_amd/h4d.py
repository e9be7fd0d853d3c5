"""ctypes binding of the C ABI in include/h4d.h (argument marshalling only).

Every computation runs in the HIP library ``libh4d.so`` next to this file;
if it is missing, or no GPU is present, the calls raise: there is no CPU
fallback.  PyTorch, when importable, only supplies the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libh4d.so")
MAX_TYPES = 8

H4D_OK, H4D_EINVAL, H4D_ENOMEM, H4D_EHIP, H4D_ECAPACITY, H4D_ENONFINITE, H4D_ENODEV = 0, -1, -2, -3, -4, -5, -6
MOVE_AUTO, MOVE_INSERT, MOVE_DELETE, MOVE_MD = 0, 1, -1, 2
PREC_FP64, PREC_FP32 = 0, 1
FLAG_EMPTY, FLAG_NONFINITE, FLAG_RETRIED, FLAG_IDLE, FLAG_INSTANT = 0x1, 0x2, 0x4, 0x8, 0x10


class H4DError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"h4d error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("n_types", C.c_int32), ("cation_type", C.c_int32), ("anion_type", C.c_int32),
        ("n_steps", C.c_int32), ("n_steps_min", C.c_int32), ("n_steps_max", C.c_int32),
        ("water", C.c_int32), ("precision", C.c_int32), ("capacity", C.c_int32),
        ("rebuild_every", C.c_int32), ("lanes_per_atom", C.c_int32), ("schedule", C.c_int32),
        ("mass", C.c_double * MAX_TYPES), ("charge", C.c_double * MAX_TYPES),
        ("sigma", C.c_double * MAX_TYPES), ("eps", C.c_double * MAX_TYPES),
        ("box", C.c_double * 3),
        ("kT", C.c_double), ("dt", C.c_double), ("w_max", C.c_double), ("kappa_sr", C.c_double),
        ("rc_lj", C.c_double), ("rc_coul", C.c_double), ("dsf_alpha", C.c_double),
        ("coulomb_k", C.c_double), ("beta_mu", C.c_double), ("lambda_s", C.c_double),
        ("skin", C.c_double), ("d_oh", C.c_double), ("d_hh", C.c_double), ("accel", C.c_double),
        ("seed", C.c_uint64), ("stream", C.c_uint64),
        ("bias_xb", C.c_double), ("bias_alpha", C.c_double),
        ("schedule_n", C.c_double),
        ("momenta", C.c_int32), ("md_refresh", C.c_double),
        ("w_max_ratio", C.c_double), ("v_ex_edge", C.c_double),
    ]


class Checkpoint(C.Structure):
    _fields_ = [
        ("params", Params), ("trial", C.c_uint64), ("md_phases", C.c_uint64), ("next_tag", C.c_int64),
        ("lanes_per_atom", C.c_int32), ("rebuild_every", C.c_int32), ("clean_trials", C.c_int32),
        ("interval_tuned", C.c_int32), ("nbr_cap", C.c_int32), ("cell_cap", C.c_int32),
        ("has_velocities", C.c_int32), ("reserved", C.c_int32),
        ("n_trials", C.c_int64), ("n_ins", C.c_int64), ("n_ins_acc", C.c_int64), ("n_del", C.c_int64),
        ("n_del_acc", C.c_int64), ("N_sum", C.c_double), ("N2_sum", C.c_double),
    ]


class Trial(C.Structure):
    _fields_ = [
        ("move", C.c_int32), ("accepted", C.c_int32), ("n_salt_before", C.c_int32),
        ("n_salt_after", C.c_int32), ("n_steps", C.c_int32), ("flags", C.c_uint32),
        ("n_atoms", C.c_int32), ("n_rebuilds", C.c_int32),
        ("trial", C.c_int64), ("tag_c", C.c_int64), ("tag_a", C.c_int64),
        ("dH", C.c_double), ("dU", C.c_double), ("dK", C.c_double), ("W_prot", C.c_double),
        ("E_switch", C.c_double), ("dM", C.c_double), ("ln_ratio", C.c_double),
        ("ln_u", C.c_double), ("ln_proposal", C.c_double), ("H0", C.c_double), ("H1", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Observables(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int64), ("n_salt", C.c_int64), ("n_trials", C.c_int64),
        ("n_ins", C.c_int64), ("n_ins_acc", C.c_int64), ("n_del", C.c_int64), ("n_del_acc", C.c_int64),
        ("U", C.c_double), ("U_lj", C.c_double), ("U_coul", C.c_double), ("virial", C.c_double),
        ("pressure_virial", C.c_double), ("N_mean", C.c_double), ("N2_mean", C.c_double),
        ("chi", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("step_launches", C.c_int64), ("retries", C.c_int64), ("step_ms", C.c_double),
                ("mean_nbr", C.c_double), ("rebuild_every", C.c_int32), ("nbr_cap", C.c_int32),
                ("lanes", C.c_int32), ("cell_cap", C.c_int32), ("atom_launches", C.c_double),
                ("nonfinite", C.c_int64), ("retries_total", C.c_int64), ("nt_lists", C.c_int32),
                ("reserved", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load libh4d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2307_11447_amd/build.py")
        # One HIP runtime per process: if PyTorch is present, let it load its
        # runtime first so that libh4d.so binds to the same libamdhip64.so.7
        # instead of pulling in a second copy.
        try:
            import torch  # noqa: F401
            torch.cuda.is_available()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.h4d_last_error.restype = C.c_char_p
        L.h4d_init_system.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64), vp, C.POINTER(vp)]
        L.h4d_build_neighbors.argtypes = [vp]
        L.h4d_run_nemd_trial.argtypes = [vp, C.c_int32, C.POINTER(Trial)]
        L.h4d_run_trials.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(Trial)]
        L.h4d_sample_observables.argtypes = [vp, C.POINTER(Observables)]
        L.h4d_get_state.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.h4d_set_trial_index.argtypes = [vp, C.c_uint64]
        L.h4d_forces_at.argtypes = [vp, C.POINTER(C.c_int32), C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        L.h4d_destroy.argtypes = [vp]
        L.h4d_set_timing.argtypes = [vp, C.c_int32]
        L.h4d_set_list_loads.argtypes = [vp, C.c_int32]
        L.h4d_stream_copy.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_double)]
        L.h4d_get_timing.argtypes = [vp, C.POINTER(Timing)]
        L.h4d_init_batch.argtypes = [C.POINTER(Params), C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), vp, C.POINTER(vp)]
        L.h4d_num_boxes.argtypes = [vp]
        L.h4d_init_speculative.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                           C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int64), vp, C.POINTER(vp)]
        L.h4d_run_speculative.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(Trial), C.POINTER(C.c_int32)]
        L.h4d_run_batch.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(Trial)]
        L.h4d_get_box_state.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.h4d_box_observables.argtypes = [vp, C.c_int32, C.POINTER(Observables)]
        L.h4d_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        fp, dp = C.POINTER(C.c_float), C.POINTER(C.c_double)
        L.h4d_mlp_create.argtypes = [C.c_uint64, vp, C.POINTER(vp)]
        L.h4d_mlp_destroy.argtypes = [vp]
        L.h4d_mlp_set_weights.argtypes = [vp, fp]
        L.h4d_mlp_get_weights.argtypes = [vp, fp]
        L.h4d_mlp_forward.argtypes = [vp, C.c_int32, fp, C.c_int32, fp]
        L.h4d_mlp_forward_static.argtypes = [vp, C.c_int32, vp, C.c_int32, vp]
        L.h4d_mlp_loss_grad.argtypes = [vp, C.c_int32, fp, fp, fp, fp]
        L.h4d_mlp_train.argtypes = [vp, C.c_int32, fp, fp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_uint64,
                                    fp]
        L.h4d_set_proposal.argtypes = [vp, vp, C.c_int32, C.c_double, C.c_double]
        L.h4d_last_site_features.argtypes = [vp, fp]
        L.h4d_last_candidates.argtypes = [vp, C.c_int32, dp, fp, fp]
        L.h4d_last_box_candidates.argtypes = [vp, C.c_int32, C.c_int32, dp, fp, fp]
        L.h4d_site_features.argtypes = [vp, C.c_int32, dp, fp]
        L.h4d_set_beta_mu.argtypes = [vp, C.c_double]
        L.h4d_set_bias.argtypes = [vp, C.c_double, C.c_double]
        L.h4d_run_md.argtypes = [vp, C.c_int32, C.POINTER(Trial)]
        L.h4d_set_early_rejection.argtypes = [vp, C.c_double]
        L.h4d_save_checkpoint.argtypes = [vp, C.POINTER(Checkpoint)]
        L.h4d_restore_checkpoint.argtypes = [vp, C.POINTER(Checkpoint), C.c_int32, dp]
        L.h4d_save_box_checkpoint.argtypes = [vp, C.c_int32, C.POINTER(Checkpoint)]
        L.h4d_restore_box_checkpoint.argtypes = [vp, C.c_int32, C.POINTER(Checkpoint), C.c_int32, dp]
        for name in ("h4d_stream_copy", "h4d_set_timing", "h4d_set_list_loads", "h4d_get_timing", "h4d_init_system", "h4d_build_neighbors",
                     "h4d_run_nemd_trial", "h4d_run_trials", "h4d_sample_observables", "h4d_get_state",
                     "h4d_set_trial_index", "h4d_forces_at", "h4d_destroy", "h4d_init_batch", "h4d_num_boxes",
                     "h4d_run_batch", "h4d_get_box_state", "h4d_box_observables", "h4d_autotune",
                     "h4d_mlp_create", "h4d_mlp_destroy", "h4d_mlp_set_weights", "h4d_mlp_get_weights",
                     "h4d_mlp_forward", "h4d_mlp_forward_static", "h4d_mlp_loss_grad", "h4d_mlp_train", "h4d_set_proposal",
                     "h4d_last_site_features", "h4d_last_candidates", "h4d_last_box_candidates", "h4d_site_features", "h4d_set_beta_mu",
                     "h4d_init_speculative", "h4d_run_speculative", "h4d_set_bias", "h4d_run_md", "h4d_set_early_rejection",
                     "h4d_save_checkpoint", "h4d_restore_checkpoint", "h4d_save_box_checkpoint",
                     "h4d_restore_box_checkpoint"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(code: int):
    if code != H4D_OK:
        raise H4DError(code, lib().h4d_last_error().decode())


def make_params(d: dict) -> Params:
    p = Params()
    p.n_types = d["n_types"]
    p.cation_type, p.anion_type = d["cation_type"], d["anion_type"]
    p.n_steps = d["n_steps"]
    p.n_steps_min, p.n_steps_max = d.get("n_steps_min", 0), d.get("n_steps_max", 0)
    p.water = d.get("water", 0)
    prec = d.get("precision", "fp64")
    p.precision = PREC_FP32 if prec in ("fp32", PREC_FP32) else PREC_FP64
    p.capacity = d.get("capacity", 0)
    p.rebuild_every = d.get("rebuild_every", 0)
    p.lanes_per_atom = d.get("lanes_per_atom", 0)
    p.bias_xb, p.bias_alpha = d.get("bias_xb", 0.0), d.get("bias_alpha", 0.0)
    p.schedule, p.schedule_n = d.get("schedule", 0), d.get("schedule_n", 1.0)
    p.momenta, p.md_refresh = d.get("momenta", 0), d.get("md_refresh", 0.0)
    p.w_max_ratio = d.get("w_max_ratio", 0.0)
    p.v_ex_edge = d.get("v_ex_edge", 0.0)
    for name in ("mass", "charge", "sigma", "eps"):
        arr = getattr(p, name)
        for i, v in enumerate(d[name]):
            arr[i] = v
    for i in range(3):
        p.box[i] = d["box"][i]
    for k in ("kT", "dt", "w_max", "kappa_sr", "rc_lj", "rc_coul", "coulomb_k", "beta_mu",
              "lambda_s", "skin", "d_oh", "d_hh"):
        setattr(p, k, d[k])
    p.dsf_alpha = d["alpha"]
    p.accel = d.get("accel", 1.0)
    p.seed, p.stream = d["seed"], d.get("stream", 0)
    return p


def current_stream():
    """The current torch HIP stream handle, or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def stream_copy(nbytes: int, reps: int = 20) -> float:
    """Mean time (ms) of a plain device copy of nbytes (read + write)."""
    ms = C.c_double()
    _check(lib().h4d_stream_copy(nbytes, reps, C.byref(ms)))
    return ms.value


N_PARAMS = 41473


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """The learned proposal's network on the GPU (64 -> 3 x 128 GELU -> 1)."""

    def __init__(self, seed: int = 0, stream=None):
        self._h = None
        h = C.c_void_p()
        _check(lib().h4d_mlp_create(seed, stream if stream is not None else current_stream(), C.byref(h)))
        self._h = h

    def close(self):
        if self._h is not None:
            lib().h4d_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32).reshape(N_PARAMS)
        _check(lib().h4d_mlp_set_weights(self._h, _fp(t)))

    def weights(self) -> np.ndarray:
        t = np.zeros(N_PARAMS, np.float32)
        _check(lib().h4d_mlp_get_weights(self._h, _fp(t)))
        return t

    def forward(self, X, bf16: bool = True) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 64)
        out = np.zeros(max(len(X), 1), np.float32)
        _check(lib().h4d_mlp_forward(self._h, len(X), _fp(X), 1 if bf16 else 0, _fp(out)))
        return out[: len(X)]

    def forward_static(self, rows: int, features_ptr: int, logits_ptr: int, bf16: bool = True):
        """h4d_mlp_forward_static: logits of rows x 64 device features into
        device memory (raw device addresses), enqueued on the network's
        stream without allocating or waiting."""
        _check(lib().h4d_mlp_forward_static(self._h, rows, C.c_void_p(features_ptr), 1 if bf16 else 0,
                                            C.c_void_p(logits_ptr)))

    def loss_grad(self, X, t):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 64)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(len(X))
        g = np.zeros(N_PARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        _check(lib().h4d_mlp_loss_grad(self._h, len(X), _fp(X), _fp(t), _fp(g), _fp(loss)))
        return float(loss[0]), g

    def train(self, X, t, steps: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
              weight_decay: float = 0.0) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 64)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(len(X))
        losses = np.zeros(max(steps, 1), np.float32)
        _check(lib().h4d_mlp_train(self._h, len(X), _fp(X), _fp(t), steps, batch, lr, weight_decay, seed,
                                   _fp(losses)))
        return losses[:steps]


def _state_of(h, box: int) -> dict:
    n = C.c_int32()
    ns = C.c_int32()
    _check(lib().h4d_get_box_state(h, box, 0, C.byref(n), C.byref(ns), None, None, None, None, None))
    cap = max(n.value, 1)
    x = np.zeros((cap, 3)); v = np.zeros((cap, 3))
    t = np.zeros(cap, np.int32); m = np.zeros(cap, np.int32)
    g = np.zeros(cap, np.int64)
    _check(lib().h4d_get_box_state(h, box, cap, C.byref(n), C.byref(ns),
                                   x.ctypes.data_as(C.POINTER(C.c_double)),
                                   v.ctypes.data_as(C.POINTER(C.c_double)),
                                   t.ctypes.data_as(C.POINTER(C.c_int32)),
                                   m.ctypes.data_as(C.POINTER(C.c_int32)),
                                   g.ctypes.data_as(C.POINTER(C.c_int64))))
    k = n.value
    return dict(n=k, nsalt=ns.value, x=x[:k], v=v[:k], type=t[:k], mol=m[:k], tag=g[:k])


class _Handle:
    """Common part of single-box systems and batches."""

    _h = None

    def close(self):
        if self._h is not None:
            lib().h4d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_neighbors(self):
        _check(lib().h4d_build_neighbors(self._h))

    def set_trial_index(self, t: int):
        _check(lib().h4d_set_trial_index(self._h, t))

    def set_bias(self, x_b: float, alpha_b: float):
        """Bimodal bias of the flying pair's separation (alpha_b = 0: off)."""
        _check(lib().h4d_set_bias(self._h, x_b, alpha_b))

    def set_early_rejection(self, v_ex_edge: float):
        """Edge of the cube V_ex around the flying cation (0: off)."""
        _check(lib().h4d_set_early_rejection(self._h, v_ex_edge))

    def set_beta_mu(self, beta_mu: float):
        _check(lib().h4d_set_beta_mu(self._h, beta_mu))

    def set_timing(self, on: bool = True):
        _check(lib().h4d_set_timing(self._h, 1 if on else 0))

    def set_list_loads(self, mode: int):
        """List-index loads of the FP32 pair pass: -1 by the list's size
        (default), 0 cached, 1 non-temporal; the results are the same."""
        _check(lib().h4d_set_list_loads(self._h, mode))

    def timing(self) -> dict:
        t = Timing()
        _check(lib().h4d_get_timing(self._h, C.byref(t)))
        return t.as_dict()

    def autotune(self, trials: int = 2):
        """Lanes per atom and base rebuild interval chosen by timing
        trials; returns (lanes, rebuild_every, ns per atom-step)."""
        lanes = C.c_int32()
        every = C.c_int32()
        ns = C.c_double()
        _check(lib().h4d_autotune(self._h, trials, C.byref(lanes), C.byref(every), C.byref(ns)))
        return lanes.value, every.value, ns.value

    def box_state(self, box: int) -> dict:
        return _state_of(self._h, box)

    def md_phase(self, n_steps: int, as_array: bool = False):
        """One equilibrium phase (generalized hybrid MC, n_steps steps) in
        every box; one record per box."""
        nb = self.n_boxes
        recs = (Trial * nb)()
        _check(lib().h4d_run_md(self._h, n_steps, recs))
        if as_array:
            return recs
        return [recs[b].as_dict() for b in range(nb)]

    def box_observables(self, box: int) -> dict:
        o = Observables()
        _check(lib().h4d_box_observables(self._h, box, C.byref(o)))
        return o.as_dict()

    def set_proposal(self, net=None, k: int = 0, cap: float = 10.0, scale: float = 1.0):
        """k <= 0: uniform proposal; k >= 1: multiple-try with k candidates
        per move and box, weighted by exp(scale * min(logit, cap)) of net
        (None: equal weights)."""
        _check(lib().h4d_set_proposal(self._h, net._h if net is not None else None, k, cap, scale))
        self._net = net     # the network must outlive its use

    def last_candidates(self, k: int, box: int = 0):
        """Sites, features and logits of the last learned move's k
        candidates in box `box`."""
        sites = np.zeros((k, 6))
        feat = np.zeros((k, 64), np.float32)
        logit = np.zeros(k, np.float32)
        rc = lib().h4d_last_box_candidates(self._h, box, k, sites.ctypes.data_as(C.POINTER(C.c_double)),
                                           _fp(feat), _fp(logit))
        if rc < 0:
            _check(rc)
        return sites, feat, logit

    @property
    def n_boxes(self) -> int:
        return lib().h4d_num_boxes(self._h)


class Batch(_Handle):
    """Independent boxes run together: box b has edges boxes[b] and its own
    Philox stream (params["stream"] + b)."""

    def __init__(self, params, boxes, xs, types, tags, nsalts, stream=None):
        """params: a dict for make_params, or a Params structure as it is."""
        self._h = None
        raw = isinstance(params, Params)
        self.params = {k: getattr(params, k) for k, _ in params._fields_} if raw else dict(params)
        nb = len(boxes)
        edges = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(nb, 3))
        n_atoms = np.array([len(t) for t in types], np.int32)
        ns = np.ascontiguousarray(nsalts, dtype=np.int32)
        x = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64).reshape(-1, 3) for v in xs]))
        t = np.ascontiguousarray(np.concatenate(types).astype(np.int32))
        g = np.ascontiguousarray(np.concatenate(tags).astype(np.int64))
        h = C.c_void_p()
        p = params if raw else make_params(params)
        _check(lib().h4d_init_batch(
            C.byref(p), nb, edges.ctypes.data_as(C.POINTER(C.c_double)),
            n_atoms.ctypes.data_as(C.POINTER(C.c_int32)), ns.ctypes.data_as(C.POINTER(C.c_int32)),
            x.ctypes.data_as(C.POINTER(C.c_double)), t.ctypes.data_as(C.POINTER(C.c_int32)),
            g.ctypes.data_as(C.POINTER(C.c_int64)),
            stream if stream is not None else current_stream(), C.byref(h)))
        self._h = h
        self.nb = nb

    @classmethod
    def from_workloads(cls, ws, **overrides):
        params = dict(ws[0].params)
        params.update(overrides)
        return cls(params, [w.params["box"] for w in ws], [w.x for w in ws], [w.type for w in ws],
                   [w.tag for w in ws], [w.nsalt for w in ws])

    def checkpoint(self) -> list:
        """One checkpoint per box (each box a chain of its own; box b's also
        resumes as a System)."""
        out = []
        for b in range(self.nb):
            ck = Checkpoint()
            _check(lib().h4d_save_box_checkpoint(self._h, b, C.byref(ck)))
            st = self.box_state(b)
            out.append({"checkpoint": np.frombuffer(bytes(ck), np.uint8).copy(), "x": st["x"], "v": st["v"],
                        "type": st["type"], "mol": st["mol"], "tag": st["tag"], "nsalt": np.int64(st["nsalt"]),
                        "n_mol": np.int64(0)})
        return out

    @classmethod
    def resume(cls, ckpts, stream=None):
        """A batch that continues every box's chain from Batch.checkpoint()."""
        cks = [_checkpoint_record(c) for c in ckpts]
        bat = cls(cks[0].params, [list(ck.params.box) for ck in cks], [c["x"] for c in ckpts],
                  [c["type"] for c in ckpts], [c["tag"] for c in ckpts], [int(c["nsalt"]) for c in ckpts],
                  stream=stream)
        try:
            for b, (ck, c) in enumerate(zip(cks, ckpts)):
                v = np.ascontiguousarray(c["v"], dtype=np.float64).reshape(-1, 3)
                _check(lib().h4d_restore_box_checkpoint(bat._h, b, C.byref(ck), len(v),
                                                        v.ctypes.data_as(C.POINTER(C.c_double))))
        except H4DError:
            bat.close()
            raise
        return bat

    def run(self, trials_per_box: int, move: int = MOVE_AUTO, as_array: bool = False):
        """trials_per_box more trials in every box; records box-major."""
        recs = (Trial * max(self.nb * trials_per_box, 1))()
        _check(lib().h4d_run_batch(self._h, trials_per_box, move, recs))
        if as_array:
            return recs
        return [[recs[b * trials_per_box + q].as_dict() for q in range(trials_per_box)] for b in range(self.nb)]


def _checkpoint_record(ckpt) -> Checkpoint:
    raw = np.ascontiguousarray(ckpt["checkpoint"], dtype=np.uint8).tobytes()
    if len(raw) != C.sizeof(Checkpoint):
        raise ValueError("checkpoint record of the wrong size")
    return Checkpoint.from_buffer_copy(raw)


def _restore(handle, ck: Checkpoint, ckpt):
    v = np.ascontiguousarray(ckpt["v"], dtype=np.float64).reshape(-1, 3)
    try:
        _check(lib().h4d_restore_checkpoint(handle._h, C.byref(ck), len(v), v.ctypes.data_as(C.POINTER(C.c_double))))
    except H4DError:
        handle.close()
        raise
    return handle


class _Chain(_Handle):
    """A single chain (one box, or speculative replicas of one box)."""

    def checkpoint(self) -> dict:
        """The chain's atoms and counters as numpy arrays (np.savez stores
        them without pickling); resume() continues the chain from them."""
        ck = Checkpoint()
        _check(lib().h4d_save_checkpoint(self._h, C.byref(ck)))
        st = self.state()
        return {"checkpoint": np.frombuffer(bytes(ck), np.uint8).copy(), "x": st["x"], "v": st["v"],
                "type": st["type"], "mol": st["mol"], "tag": st["tag"], "nsalt": np.int64(st["nsalt"]),
                "n_mol": np.int64(self.n_mol)}


class Speculative(_Chain):
    """One chain run speculatively on `replicas` copies of its state: a
    round runs the next `replicas` trials side by side and keeps them up to
    the first accepted one (the records equal a one-by-one run)."""

    def __init__(self, params, replicas: int, x, type_, mol, tag, nsalt: int, n_mol: int = 0, stream=None):
        """params: a dict for make_params, or a Params structure as it is."""
        self._h = None
        raw = isinstance(params, Params)
        self.params = {k: getattr(params, k) for k, _ in params._fields_} if raw else dict(params)
        self.n_mol = n_mol
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(type_, dtype=np.int32)
        m = np.ascontiguousarray(mol, dtype=np.int32)
        g = np.ascontiguousarray(tag, dtype=np.int64)
        h = C.c_void_p()
        p = params if raw else make_params(params)
        _check(lib().h4d_init_speculative(
            C.byref(p), replicas, len(t), nsalt, n_mol, x.ctypes.data_as(C.POINTER(C.c_double)),
            t.ctypes.data_as(C.POINTER(C.c_int32)), m.ctypes.data_as(C.POINTER(C.c_int32)),
            g.ctypes.data_as(C.POINTER(C.c_int64)), stream if stream is not None else current_stream(), C.byref(h)))
        self._h = h
        self.replicas = replicas
        self.rounds = 0

    @classmethod
    def resume(cls, ckpt, replicas: int, stream=None):
        """Speculative replicas that continue the chain saved by checkpoint()
        (of a System or of a Speculative handle)."""
        ck = _checkpoint_record(ckpt)
        return _restore(cls(ck.params, replicas, ckpt["x"], ckpt["type"], ckpt["mol"], ckpt["tag"],
                            int(ckpt["nsalt"]), int(ckpt["n_mol"]), stream=stream), ck, ckpt)

    @classmethod
    def from_workload(cls, w, replicas: int, **overrides):
        params = dict(w.params)
        params.update(overrides)
        return cls(params, replicas, w.x, w.type, w.mol, w.tag, w.nsalt, n_mol=w.n_mol)

    def trials(self, n: int, move: int = MOVE_AUTO, as_array: bool = False):
        recs = (Trial * max(n, 1))()
        rounds = C.c_int32()
        _check(lib().h4d_run_speculative(self._h, n, move, recs, C.byref(rounds)))
        self.rounds += rounds.value
        if as_array:
            return recs
        return [recs[q].as_dict() for q in range(n)]

    def state(self) -> dict:
        return _state_of(self._h, 0)


class System(_Chain):
    """One simulation box on the GPU."""

    def __init__(self, params, x, type_, mol, tag, nsalt: int, n_mol: int = 0, stream=None):
        """params: a dict for make_params, or a Params structure as it is."""
        self._h = None
        raw = isinstance(params, Params)
        self.params = {k: getattr(params, k) for k, _ in params._fields_} if raw else dict(params)
        self.n_mol = n_mol
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(type_, dtype=np.int32)
        m = np.ascontiguousarray(mol, dtype=np.int32)
        g = np.ascontiguousarray(tag, dtype=np.int64)
        h = C.c_void_p()
        p = params if raw else make_params(params)
        _check(lib().h4d_init_system(
            C.byref(p), len(t), nsalt, n_mol,
            x.ctypes.data_as(C.POINTER(C.c_double)), t.ctypes.data_as(C.POINTER(C.c_int32)),
            m.ctypes.data_as(C.POINTER(C.c_int32)), g.ctypes.data_as(C.POINTER(C.c_int64)),
            stream if stream is not None else current_stream(), C.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, w, **overrides):
        params = dict(w.params)
        params.update(overrides)
        return cls(params, w.x, w.type, w.mol, w.tag, w.nsalt, w.n_mol)

    @classmethod
    def resume(cls, ckpt, stream=None):
        """A new handle that continues the chain saved by checkpoint() (of a
        System or of a Speculative handle)."""
        ck = _checkpoint_record(ckpt)
        return _restore(cls(ck.params, ckpt["x"], ckpt["type"], ckpt["mol"], ckpt["tag"], int(ckpt["nsalt"]),
                            int(ckpt["n_mol"]), stream=stream), ck, ckpt)

    def trial(self, move: int = MOVE_AUTO) -> dict:
        r = Trial()
        _check(lib().h4d_run_nemd_trial(self._h, move, C.byref(r)))
        return r.as_dict()


    def trials(self, n: int, move: int = MOVE_AUTO, as_array: bool = False):
        recs = (Trial * max(n, 1))()
        _check(lib().h4d_run_trials(self._h, n, move, recs))
        if as_array:
            return recs
        return [recs[q].as_dict() for q in range(n)]

    def state(self) -> dict:
        return _state_of(self._h, 0)

    def forces_at(self, flying=(-1, -1), w: float = 0.0):
        st = self.state()
        F = np.zeros((max(st["n"], 1), 3))
        e = np.zeros(3)
        fl = (C.c_int32 * 2)(*flying)
        _check(lib().h4d_forces_at(self._h, fl, w, F.ctypes.data_as(C.POINTER(C.c_double)),
                                   e.ctypes.data_as(C.POINTER(C.c_double))))
        return F[: st["n"]], dict(U=e[0], U_lj=e[1], U_c=e[2])

    def last_site_features(self) -> np.ndarray:
        f = np.zeros(64, np.float32)
        _check(lib().h4d_last_site_features(self._h, _fp(f)))
        return f

    def site_features(self, sites) -> np.ndarray:
        st = np.ascontiguousarray(sites, dtype=np.float64).reshape(-1, 6)
        out = np.zeros((len(st), 64), np.float32)
        _check(lib().h4d_site_features(self._h, len(st), st.ctypes.data_as(C.POINTER(C.c_double)), _fp(out)))
        return out

    def observables(self) -> dict:
        o = Observables()
        _check(lib().h4d_sample_observables(self._h, C.byref(o)))
        return o.as_dict()
