"""Python binding of the C ABI in ``include/tkdv.h`` (ctypes; argument marshalling only).

Every step of the sampler runs in the HIP library ``libtkdv.so``; PyTorch is
used here only to allocate device memory and to pass the current HIP stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtkdv.so")

KMAX = 128
NBINS = 64

UNIFORM, SIGMA, MIXTURE = 0, 1, 2
MV_RAISE, MV_FAIL, MV_COUNT = 0, 1, 2   # policies for proposals with f/(M g) > 1
MIX_S, MIX_R = 32, 2
FP32, BF16, BF16X3 = 0, 1, 2
COUNT_PROPOSALS, COUNT_ACCEPTED = 0, 1

PRECISIONS = {"fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}
PROPOSALS = {"uniform": UNIFORM, "sigma": SIGMA, "mixture": MIXTURE}

STATUS = {0: "ok", -1: "invalid argument", -2: "no alpha root", -3: "HIP error",
          -4: "capacity exceeded", -5: "unsupported K", -6: "M violation"}


class TkdvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tkdv status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Point(C.Structure):
    _fields_ = [("K", C.c_int32), ("point_id", C.c_uint32), ("E0", C.c_double),
                ("beta_p", C.c_double), ("c32", C.c_double), ("seed", C.c_uint64)]


PLAN_SEARCH_ALWAYS = 1  # tkdv_plan_batch: search also where C3/C2 = 0


class Plan(C.Structure):
    _fields_ = [("alpha_star", C.c_double), ("log_M", C.c_double), ("log_norm_g", C.c_double),
                ("sigma2", C.c_double * KMAX), ("N", C.c_int32), ("proposal", C.c_int32),
                ("M_source", C.c_int32), ("n_optimiser_evals", C.c_int32)]


class SirStats(C.Structure):
    """Result of tkdv_sir."""
    _fields_ = [("n", C.c_uint64), ("m", C.c_uint64), ("n_over_one", C.c_uint64), ("pad", C.c_uint64),
                ("W", C.c_double), ("W2", C.c_double), ("ess", C.c_double), ("max_w", C.c_double),
                ("mean", C.c_double), ("m2", C.c_double), ("m3", C.c_double), ("m4", C.c_double),
                ("skewness", C.c_double), ("kurtosis", C.c_double)]

    def to_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class Mixture(C.Structure):
    """Learned defensive mixture (tkdv_mixture): base ACG L0 = D + V V^T and its S shifts."""
    _fields_ = [("K", C.c_int32), ("pad", C.c_int32), ("eps", C.c_double),
                ("logd", C.c_double * KMAX), ("V", (C.c_double * MIX_R) * (2 * KMAX))]


class LaunchCfg(C.Structure):
    """Launch configuration of the sweep (tkdv_launch_cfg)."""
    _fields_ = [("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32), ("window", C.c_uint64),
                ("variant", C.c_int32), ("adaptive", C.c_int32)]

    def __init__(self, blocks_per_cu: int = 0, use_graph: int = 1, window: int = 1 << 26, variant: int = 0,
                 adaptive: int = 1):
        super().__init__(int(blocks_per_cu), int(use_graph), int(window), int(variant), int(adaptive))

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class LearnerCfg(C.Structure):
    _fields_ = [("K", C.c_int32), ("hidden", C.c_int32), ("eps", C.c_double), ("v_amp", C.c_double),
                ("v_scale", C.c_double), ("temperature", C.c_double), ("nll_weight", C.c_double),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("seed", C.c_uint64)]


class Timing(C.Structure):
    _fields_ = [("decide_ms", C.c_double), ("fixup_ms", C.c_double), ("segments_ms", C.c_double),
                ("materialize_ms", C.c_double), ("finalize_ms", C.c_double), ("synth_ms", C.c_double),
                ("total_ms", C.c_double),
                ("decide_launches", C.c_int32), ("decide_grid", C.c_int32), ("decide_block", C.c_int32),
                ("windows", C.c_int32), ("graph_launches", C.c_int32)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MapCell(C.Structure):
    _fields_ = [("beta_p", C.c_double), ("c32", C.c_double), ("alpha_star", C.c_double), ("log_M", C.c_double),
                ("n_proposed", C.c_uint64), ("n_accepted", C.c_uint64), ("acceptance", C.c_double),
                ("skewness", C.c_double), ("kurtosis", C.c_double), ("p_exceed_2sigma", C.c_double),
                ("p_exceed_4sigma", C.c_double), ("p_sample_4sigma", C.c_double), ("peak_u", C.c_double),
                ("peak_index", C.c_uint64), ("status", C.c_int32), ("M_raises", C.c_int32)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


MAP_MAX_CELLS = 4096


class Stats(C.Structure):
    _fields_ = [("n_proposed", C.c_uint64), ("n_accepted", C.c_uint64), ("n_written", C.c_uint64),
                ("n_fp64_fixups", C.c_uint64), ("n_M_violations", C.c_uint64),
                ("n_exceed_2sigma", C.c_uint64), ("n_grid_values", C.c_uint64),
                ("max_log_a", C.c_double), ("S1", C.c_double), ("S2", C.c_double),
                ("S3", C.c_double), ("S4", C.c_double), ("skewness", C.c_double),
                ("kurtosis", C.c_double), ("p_exceed_2sigma", C.c_double),
                ("hist_lo", C.c_double), ("hist_hi", C.c_double),
                ("hist_u0", C.c_uint64 * NBINS), ("log_M_used", C.c_double), ("M_raises", C.c_int32),
                ("fallback", C.c_int32), ("n_exceed_4sigma", C.c_uint64), ("n_samples_4sigma", C.c_uint64),
                ("peak_u", C.c_double), ("peak_index", C.c_uint64)]

    def to_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "hist_u0"}
        d["hist_u0"] = np.array(self.hist_u0[:], dtype=np.uint64)
        d["acceptance"] = self.n_accepted / self.n_proposed if self.n_proposed else float("nan")
        return d


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_16952_amd.build` "
                          "(or __graft_entry__.build()) before using the GPU sampler")
    return C.CDLL(LIB_PATH)


lib = _load()

EXPORTS = ["tkdv_create", "tkdv_destroy", "tkdv_plan_point", "tkdv_sample", "tkdv_sample_batch",
           "tkdv_eval_proposals", "tkdv_synthesize", "tkdv_decision_window", "tkdv_get_timing",
           "tkdv_status_str", "tkdv_last_error", "tkdv_mixture_log_q", "tkdv_plan_mixture",
           "tkdv_sample_mixture", "tkdv_eval_mixture", "tkdv_mixture_window", "tkdv_learner_create",
           "tkdv_learner_destroy", "tkdv_learner_set_points", "tkdv_learner_add_rows",
           "tkdv_learner_add_rows_host", "tkdv_learner_add_shifted_rows", "tkdv_learner_train",
           "tkdv_learner_gradients",
           "tkdv_learner_mixture", "tkdv_learner_n_weights", "tkdv_learner_get_weights",
           "tkdv_learner_set_weights", "tkdv_sample_sweep", "tkdv_set_launch_cfg", "tkdv_get_launch_cfg",
           "tkdv_autotune", "tkdv_plan_batch", "tkdv_extremes", "tkdv_sir", "tkdv_plan_mixture_batch",
           "tkdv_set_violation_policy", "tkdv_sample_noalloc", "tkdv_extremes_map"]

_P = C.c_void_p
lib.tkdv_create.argtypes = [C.c_int, C.POINTER(_P)]
lib.tkdv_destroy.argtypes = [_P]
lib.tkdv_plan_point.argtypes = [C.POINTER(Point), C.c_int, C.POINTER(Plan)]
lib.tkdv_sample.argtypes = [_P, C.POINTER(Point), C.c_int, C.POINTER(Plan), C.c_uint64, C.c_int,
                            C.c_uint64, C.c_int, _P, _P, C.c_uint64, C.POINTER(Stats), _P]
lib.tkdv_sample_noalloc.argtypes = [_P, C.POINTER(Point), C.c_int, C.POINTER(Plan), C.c_uint64, C.c_int,
                                    C.c_uint64, C.c_int, _P, _P, C.c_uint64, C.POINTER(Stats), _P]
lib.tkdv_sample_batch.argtypes = [_P, C.c_int32, C.POINTER(Point), C.c_int, C.POINTER(Plan),
                                  C.POINTER(C.c_uint64), C.c_int, C.c_uint64, C.c_int, _P, _P,
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(Stats), _P]
lib.tkdv_eval_proposals.argtypes = [_P, C.POINTER(Point), C.c_int, C.POINTER(Plan), C.c_uint64,
                                    C.c_uint64, C.c_int, _P, _P, _P, _P, _P, _P, _P]
lib.tkdv_get_timing.argtypes = [_P, C.POINTER(Timing)]
lib.tkdv_set_violation_policy.argtypes = [_P, C.c_int]
lib.tkdv_synthesize.argtypes = [_P, C.c_int32, C.c_int, _P, C.c_uint64, _P, _P]
lib.tkdv_decision_window.argtypes = [C.POINTER(Point), C.c_int, C.c_int]
lib.tkdv_decision_window.restype = C.c_double
_PD = C.POINTER(C.c_double)
lib.tkdv_mixture_log_q.argtypes = [C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture), _PD, C.c_int32, _PD, _PD]
lib.tkdv_plan_mixture.argtypes = [C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture), _PD, C.c_int32,
                                  C.c_double, C.POINTER(Plan), _PD]
lib.tkdv_sample_mixture.argtypes = [_P, C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture), C.c_uint64,
                                    C.c_int, C.c_uint64, C.c_int, _P, _P, C.c_uint64, C.POINTER(Stats), _P]
lib.tkdv_eval_mixture.argtypes = [_P, C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture), C.c_uint64,
                                  C.c_uint64, C.c_int, _P, _P, _P, _P, _P, _P, _P]
lib.tkdv_mixture_window.argtypes = [C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture), C.c_int]
lib.tkdv_mixture_window.restype = C.c_double
lib.tkdv_learner_create.argtypes = [_P, C.POINTER(LearnerCfg), C.POINTER(_P)]
lib.tkdv_learner_destroy.argtypes = [_P]
lib.tkdv_learner_set_points.argtypes = [_P, C.c_int32, C.POINTER(Point), C.POINTER(Plan)]
lib.tkdv_learner_add_rows.argtypes = [_P, C.c_int32, _P, C.c_uint64, C.c_uint64, C.c_int32, _P]
lib.tkdv_learner_add_rows_host.argtypes = [_P, C.c_int32, _PD, C.c_uint64, C.c_int32]
lib.tkdv_learner_add_shifted_rows.argtypes = [_P, C.c_int32, _PD, C.c_uint64, _PD, C.c_int32, C.c_int32]
lib.tkdv_learner_train.argtypes = [_P, C.c_int32, _PD, _P]
lib.tkdv_learner_gradients.argtypes = [_P, _PD, _PD, _PD, _P]
lib.tkdv_learner_mixture.argtypes = [_P, C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture)]
lib.tkdv_learner_n_weights.argtypes = [_P]
lib.tkdv_learner_n_weights.restype = C.c_int64
lib.tkdv_learner_get_weights.argtypes = [_P, _PD, C.c_int64]
lib.tkdv_learner_set_weights.argtypes = [_P, _PD, C.c_int64]
lib.tkdv_sample_sweep.argtypes = [_P, C.c_int32, C.POINTER(Point), C.POINTER(Plan), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_uint64), C.c_int, C.POINTER(LaunchCfg), _P, _P,
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(Stats), _P]
lib.tkdv_set_launch_cfg.argtypes = [_P, C.c_int32, C.c_int, C.POINTER(LaunchCfg)]
lib.tkdv_get_launch_cfg.argtypes = [_P, C.c_int32, C.c_int, C.POINTER(LaunchCfg)]
lib.tkdv_autotune.argtypes = [_P, C.c_int32, C.c_int, C.c_char_p, C.POINTER(LaunchCfg)]
lib.tkdv_extremes.argtypes = [_P, C.c_int32, C.c_double, _P, C.c_uint64, C.c_uint64, C.c_int32, C.c_double,
                              C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                              C.POINTER(C.c_uint64), _P, _P, _P]
lib.tkdv_sir.argtypes = [_P, C.POINTER(Point), C.c_int, C.POINTER(Plan), C.c_uint64, C.c_uint64, C.c_double,
                         C.c_int, _P, _P, _P, C.POINTER(SirStats), _P]
lib.tkdv_plan_mixture_batch.argtypes = [_P, C.c_int32, C.POINTER(Point), C.POINTER(Plan), C.POINTER(Mixture),
                                        C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_uint64, C.c_double,
                                        C.POINTER(Plan), C.POINTER(C.c_double), _P]
lib.tkdv_plan_batch.argtypes = [_P, C.c_int32, C.POINTER(Point), C.c_int, C.c_int32, C.c_uint64, C.c_int32,
                                C.POINTER(Plan), C.POINTER(C.c_double), _P]
lib.tkdv_extremes_map.argtypes = [_P, C.c_int32, C.c_double, C.c_int32, _PD, C.c_int32, _PD, C.c_uint64,
                                  C.c_uint32, C.c_uint64, C.c_uint64, C.c_int, C.POINTER(MapCell), _P]
lib.tkdv_status_str.argtypes = [C.c_int]
lib.tkdv_status_str.restype = C.c_char_p
lib.tkdv_last_error.argtypes = [_P]
lib.tkdv_last_error.restype = C.c_char_p
for _f in EXPORTS:
    if _f not in ("tkdv_decision_window", "tkdv_status_str", "tkdv_last_error", "tkdv_mixture_window",
                  "tkdv_learner_n_weights"):
        getattr(lib, _f).restype = C.c_int


def _check(st: int, ctx=None):
    if st != 0:
        msg = lib.tkdv_last_error(ctx)
        raise TkdvError(st, msg.decode() if msg else "")


def make_point(K: int, E0: float, beta_p: float, c32: float, seed: int = 0, point_id: int = 0) -> Point:
    return Point(int(K), int(point_id), float(E0), float(beta_p), float(c32), int(seed))


def plan_point(point: Point, proposal: int = SIGMA) -> Plan:
    pl = Plan()
    _check(lib.tkdv_plan_point(C.byref(point), int(proposal), C.byref(pl)))
    return pl


def decision_window(point: Point, proposal: int, precision: int) -> float:
    return lib.tkdv_decision_window(C.byref(point), int(proposal), int(precision))


def make_mixture(K: int, eps: float, logd, V) -> Mixture:
    """tkdv_mixture from log d [K] and V [2K, 2] (host arrays)."""
    m = Mixture()
    m.K, m.eps = int(K), float(eps)
    logd = np.asarray(logd, dtype=np.float64).reshape(K)
    V = np.asarray(V, dtype=np.float64).reshape(2 * K, MIX_R)
    for k in range(K):
        m.logd[k] = logd[k]
    for c in range(2 * K):
        for q in range(MIX_R):
            m.V[c][q] = V[c, q]
    return m


def mixture_log_q(point: Point, sigma_plan: Plan, mix: Mixture, xhat) -> tuple[np.ndarray, np.ndarray]:
    """Host FP64 (log q_net, log q_mix) at rows x^ of shape (n, 2K)."""
    x = np.ascontiguousarray(np.asarray(xhat, dtype=np.float64).reshape(-1, 2 * point.K))
    n = x.shape[0]
    a, b = np.zeros(n), np.zeros(n)
    _check(lib.tkdv_mixture_log_q(C.byref(point), C.byref(sigma_plan), C.byref(mix),
                                  x.ctypes.data_as(_PD), n, a.ctypes.data_as(_PD), b.ctypes.data_as(_PD)))
    return a, b


def plan_mixture(point: Point, sigma_plan: Plan, mix: Mixture, starts=None, margin: float = 0.0):
    """(plan with log M_mix, argmax) by multi-start BFGS on the sphere."""
    K = point.K
    st = None if starts is None else np.ascontiguousarray(np.asarray(starts, dtype=np.float64).reshape(-1, 2 * K))
    out = Plan()
    am = np.zeros(2 * K)
    _check(lib.tkdv_plan_mixture(C.byref(point), C.byref(sigma_plan), C.byref(mix),
                                 st.ctypes.data_as(_PD) if st is not None else None,
                                 0 if st is None else st.shape[0], float(margin), C.byref(out),
                                 am.ctypes.data_as(_PD)))
    return out, am


def mixture_window(point: Point, mix_plan: Plan, mix: Mixture, precision: int) -> float:
    return lib.tkdv_mixture_window(C.byref(point), C.byref(mix_plan), C.byref(mix), int(precision))


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A sampler context on one HIP device (workspaces and synthesis tables)."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        _check(lib.tkdv_create(int(device), C.byref(self._h)))
        self.device = device

    def close(self):
        if self._h:
            lib.tkdv_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_violation_policy(self, policy: int):
        """MV_RAISE (raise M and run again; default), MV_FAIL or MV_COUNT."""
        _check(lib.tkdv_set_violation_policy(self._h, int(policy)), self._h)

    def timing(self) -> dict:
        """Device time of the phases of the last call (HIP events on its stream)."""
        t = Timing()
        _check(lib.tkdv_get_timing(self._h, C.byref(t)), self._h)
        return t.to_dict()

    def sample(self, point: Point, n: int, proposal: int = SIGMA, plan: Plan | None = None,
               mode: int = COUNT_PROPOSALS, max_proposals: int = 0, precision: int = BF16X3,
               capacity: int = 0, xhat=None, index=None, stream=None) -> dict:
        """Rejection-sample one point; returns stats (dict) plus the output tensors."""
        import torch
        dev = torch.device("cuda", self.device)
        if capacity and xhat is None:
            xhat = torch.empty((capacity, 2 * point.K), dtype=torch.float32, device=dev)
        if capacity and index is None:
            index = torch.empty((capacity,), dtype=torch.int64, device=dev)
        st = Stats()
        _check(lib.tkdv_sample(self._h, C.byref(point), int(proposal),
                               C.byref(plan) if plan is not None else None, int(n), int(mode),
                               int(max_proposals), int(precision), _ptr(xhat), _ptr(index),
                               int(capacity), C.byref(st), _stream(stream)), self._h)
        d = st.to_dict()
        nw = d["n_written"]
        d["xhat"] = xhat[:nw] if xhat is not None else None
        d["index"] = index[:nw] if index is not None else None
        return d

    def sample_noalloc(self, point: Point, n: int, plan: Plan, proposal: int = SIGMA,
                       mode: int = COUNT_PROPOSALS, max_proposals: int = 0, precision: int = BF16X3,
                       xhat=None, index=None, stream=None) -> dict:
        """tkdv_sample_noalloc: the library allocates nothing; the caller passes
        the output tensors (xhat (capacity, 2K) float32, index (capacity,) int64,
        both or neither), the plan is required."""
        assert (xhat is None) == (index is None)
        capacity = 0 if xhat is None else int(xhat.shape[0])
        st = Stats()
        _check(lib.tkdv_sample_noalloc(self._h, C.byref(point), int(proposal), C.byref(plan), int(n), int(mode),
                                       int(max_proposals), int(precision), _ptr(xhat), _ptr(index), capacity,
                                       C.byref(st), _stream(stream)), self._h)
        d = st.to_dict()
        nw = d["n_written"]
        d["xhat"] = xhat[:nw] if xhat is not None else None
        d["index"] = index[:nw] if index is not None else None
        return d

    def sample_mixture(self, point: Point, plan: Plan, mix: Mixture, n: int, mode: int = COUNT_PROPOSALS,
                       max_proposals: int = 0, precision: int = BF16X3, capacity: int = 0, xhat=None,
                       index=None, stream=None) -> dict:
        """Rejection-sample one point with the learned mixture proposal."""
        import torch
        dev = torch.device("cuda", self.device)
        if capacity and xhat is None:
            xhat = torch.empty((capacity, 2 * point.K), dtype=torch.float32, device=dev)
        if capacity and index is None:
            index = torch.empty((capacity,), dtype=torch.int64, device=dev)
        st = Stats()
        _check(lib.tkdv_sample_mixture(self._h, C.byref(point), C.byref(plan), C.byref(mix), int(n), int(mode),
                                       int(max_proposals), int(precision), _ptr(xhat), _ptr(index),
                                       int(capacity), C.byref(st), _stream(stream)), self._h)
        d = st.to_dict()
        nw = d["n_written"]
        d["xhat"] = xhat[:nw] if xhat is not None else None
        d["index"] = index[:nw] if index is not None else None
        return d

    def eval_mixture(self, point: Point, plan: Plan, mix: Mixture, i0: int, n: int,
                     precision: int = BF16X3, stream=None) -> dict:
        """eval_proposals for the learned mixture proposal."""
        import torch
        dev = torch.device("cuda", self.device)
        K = point.K
        out = {
            "xhat": torch.empty((n, 2 * K), dtype=torch.float32, device=dev),
            "t": torch.empty((n,), dtype=torch.float32, device=dev),
            "s3": torch.empty((n,), dtype=torch.float32, device=dev),
            "log_a": torch.empty((n,), dtype=torch.float32, device=dev),
            "log_u": torch.empty((n,), dtype=torch.float32, device=dev),
            "accept": torch.empty((n,), dtype=torch.uint8, device=dev),
        }
        _check(lib.tkdv_eval_mixture(self._h, C.byref(point), C.byref(plan), C.byref(mix), int(i0), int(n),
                                     int(precision), _ptr(out["xhat"]), _ptr(out["t"]), _ptr(out["s3"]),
                                     _ptr(out["log_a"]), _ptr(out["log_u"]), _ptr(out["accept"]),
                                     _stream(stream)), self._h)
        return out

    def sample_batch(self, points: list, n: list, proposal: int = SIGMA, plans: list | None = None,
                     mode: int = COUNT_PROPOSALS, max_proposals: int = 0, precision: int = BF16X3,
                     capacity: list | None = None, stream=None) -> tuple[list, object, object]:
        """Many points in one launch sequence; rows have stride 2*KMAX floats."""
        import torch
        npnt = len(points)
        pts = (Point * npnt)(*points)
        pls = (Plan * npnt)(*plans) if plans is not None else None
        nn = (C.c_uint64 * npnt)(*[int(v) for v in n])
        cap = [int(c) for c in (capacity or [0] * npnt)]
        offs = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
        total = int(sum(cap))
        dev = torch.device("cuda", self.device)
        xhat = torch.empty((max(total, 1), 2 * KMAX), dtype=torch.float32, device=dev)
        index = torch.empty((max(total, 1),), dtype=torch.int64, device=dev)
        caps = (C.c_uint64 * npnt)(*cap)
        offc = (C.c_uint64 * npnt)(*[int(v) for v in offs])
        sts = (Stats * npnt)()
        _check(lib.tkdv_sample_batch(self._h, npnt, pts, int(proposal), pls, nn, int(mode),
                                     int(max_proposals), int(precision), _ptr(xhat), _ptr(index),
                                     caps, offc, sts, _stream(stream)), self._h)
        out = []
        for p in range(npnt):
            d = sts[p].to_dict()
            o, nw = int(offs[p]), d["n_written"]
            d["xhat"] = xhat[o:o + nw, : 2 * points[p].K]
            d["index"] = index[o:o + nw]
            out.append(d)
        return out, xhat, index

    def sample_sweep(self, points: list, targets: list, max_proposals: list, plans: list | None = None,
                     precision: int = BF16X3, cfg: LaunchCfg | None = None, capacity: list | None = None,
                     stream=None) -> tuple[list, object, object]:
        """Accepted-count sweep of many points (windows replayed as a hipGraph);
        rows have stride 2*KMAX floats."""
        import torch
        npnt = len(points)
        pts = (Point * npnt)(*points)
        pls = (Plan * npnt)(*plans) if plans is not None else None
        tg = (C.c_uint64 * npnt)(*[int(v) for v in targets])
        mp = (C.c_uint64 * npnt)(*[int(v) for v in max_proposals])
        cap = [int(c) for c in (capacity or [0] * npnt)]
        offs = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
        total = int(sum(cap))
        dev = torch.device("cuda", self.device)
        xhat = torch.empty((max(total, 1), 2 * KMAX), dtype=torch.float32, device=dev)
        index = torch.empty((max(total, 1),), dtype=torch.int64, device=dev)
        caps = (C.c_uint64 * npnt)(*cap)
        offc = (C.c_uint64 * npnt)(*[int(v) for v in offs])
        sts = (Stats * npnt)()
        _check(lib.tkdv_sample_sweep(self._h, npnt, pts, pls, tg, mp, int(precision),
                                     C.byref(cfg) if cfg is not None else None, _ptr(xhat), _ptr(index),
                                     caps, offc, sts, _stream(stream)), self._h)
        out = []
        for p in range(npnt):
            d = sts[p].to_dict()
            o, nw = int(offs[p]), d["n_written"]
            d["xhat"] = xhat[o:o + nw, : 2 * points[p].K]
            d["index"] = index[o:o + nw]
            out.append(d)
        return out, xhat, index

    def extremes_map(self, K: int, E0: float, betas, c32s, n_accepted: int, max_proposals: int, seed: int = 0,
                     point_id0: int = 0, precision: int = BF16X3, stream=None) -> list:
        """Extremes over a (beta', C3/C2) grid (tkdv_extremes_map): one dict per
        cell, row-major over betas x c32s."""
        b = np.ascontiguousarray(betas, dtype=np.float64)
        c = np.ascontiguousarray(c32s, dtype=np.float64)
        cells = (MapCell * max(b.size * c.size, 1))()
        _check(lib.tkdv_extremes_map(self._h, int(K), float(E0), b.size, b.ctypes.data_as(_PD), c.size,
                                     c.ctypes.data_as(_PD), int(seed), int(point_id0), int(n_accepted),
                                     int(max_proposals), int(precision), cells, _stream(stream)), self._h)
        return [cells[q].to_dict() for q in range(b.size * c.size)]

    def set_launch_cfg(self, K: int, precision: int, cfg: LaunchCfg):
        _check(lib.tkdv_set_launch_cfg(self._h, int(K), int(precision), C.byref(cfg)), self._h)

    def get_launch_cfg(self, K: int, precision: int) -> LaunchCfg:
        c = LaunchCfg()
        _check(lib.tkdv_get_launch_cfg(self._h, int(K), int(precision), C.byref(c)), self._h)
        return c

    def autotune(self, K: int, precision: int = BF16X3, cache_path: str | None = None) -> LaunchCfg:
        c = LaunchCfg()
        _check(lib.tkdv_autotune(self._h, int(K), int(precision),
                                 cache_path.encode() if cache_path else None, C.byref(c)), self._h)
        return c

    def plan_batch(self, points: list, proposal: int = SIGMA, n_starts: int = 16, seed: int = 0,
                   search_always: bool = False, stream=None) -> tuple[list, np.ndarray]:
        """Plans of many points with log M searched on the GPU (tkdv_plan_batch):
        (plans, maximisers [n, 2K_max])."""
        n = len(points)
        pts = (Point * max(n, 1))(*points)
        plans = (Plan * max(n, 1))()
        xb = np.zeros((max(n, 1), 2 * KMAX))
        _check(lib.tkdv_plan_batch(self._h, n, pts, int(proposal), int(n_starts), int(seed),
                                   PLAN_SEARCH_ALWAYS if search_always else 0, plans,
                                   xb.ctypes.data_as(C.POINTER(C.c_double)),
                                   _stream(stream) if n else None), self._h)
        return [plans[i] for i in range(n)], xb[:n]

    def plan_mixture_batch(self, points: list, sigma_plans: list, mixes: list, starts=None, n_starts: int = 16,
                           seed: int = 0, margin: float = 0.0, stream=None) -> tuple[list, np.ndarray]:
        """log M_mix of many points searched on the GPU (tkdv_plan_mixture_batch):
        (mixture plans, maximisers [n, 2K_max]).  starts: None or an array
        (n, n_user, 2K) of caller starts per point."""
        n = len(points)
        pts = (Point * max(n, 1))(*points)
        sps = (Plan * max(n, 1))(*sigma_plans)
        mxs = (Mixture * max(n, 1))(*mixes)
        n_user = 0
        st = None
        if starts is not None:
            a = np.asarray(starts, dtype=np.float64)
            n_user = a.shape[1]
            st = np.zeros((n, n_user, 2 * KMAX))
            st[:, :, :a.shape[2]] = a
            st = np.ascontiguousarray(st)
        out = (Plan * max(n, 1))()
        xb = np.zeros((max(n, 1), 2 * KMAX))
        _check(lib.tkdv_plan_mixture_batch(self._h, n, pts, sps, mxs,
                                           st.ctypes.data_as(C.POINTER(C.c_double)) if st is not None else None,
                                           n_user, int(n_starts), int(seed), float(margin), out,
                                           xb.ctypes.data_as(C.POINTER(C.c_double)),
                                           _stream(stream) if n else None), self._h)
        return [out[i] for i in range(n)], xb[:n]

    def extremes(self, xhat, K: int, E0: float = 1.0, top_k: int = 10, threshold: float | None = None,
                 per_row: bool = False, stream=None) -> dict:
        """Largest surface displacements among rows x^ (tkdv_extremes): the top_k rows
        by max_j u(xi_j) (descending, ties by lower row), their maxima and grid
        indices, and the number of rows whose maximum exceeds `threshold`
        (default 4 sigma = 4 sqrt(E0/pi)).  xhat: float32 device tensor (n, >= 2K)
        with unit column stride."""
        import torch
        assert xhat.dtype == torch.float32 and xhat.dim() == 2 and (xhat.shape[0] == 0 or xhat.stride(1) == 1)
        n = int(xhat.shape[0])
        stride = int(xhat.stride(0)) if n else 2 * K
        thr = 4.0 * math.sqrt(E0 / math.pi) if threshold is None else float(threshold)
        kk = max(int(top_k), 1)
        rows = (C.c_uint64 * kk)()
        um = (C.c_double * kk)()
        jm = (C.c_int32 * kk)()
        nex = C.c_uint64()
        du = dj = None
        if per_row:
            du = torch.empty((n,), dtype=torch.float32, device=xhat.device)
            dj = torch.empty((n,), dtype=torch.int32, device=xhat.device)
        _check(lib.tkdv_extremes(self._h, int(K), float(E0), _ptr(xhat) if n else None, n, stride, int(top_k), thr,
                                 rows, um, jm, C.byref(nex), _ptr(du) if n else None, _ptr(dj) if n else None,
                                 _stream(stream)), self._h)
        k = min(int(top_k), n)
        return {"rows": np.array(rows[:k], dtype=np.uint64), "umax": np.array(um[:k]),
                "jmax": np.array(jm[:k], dtype=np.int64), "n_exceed": int(nex.value), "threshold": thr,
                "umax_rows": du, "jmax_rows": dj}

    def sir(self, point: Point, n: int, m: int, u0: float = 0.5, proposal: int = SIGMA, plan: Plan | None = None,
            precision: int = BF16X3, rows: bool = False, weights: bool = False, stream=None) -> dict:
        """Sampling-importance resampling over proposals 0..n-1 (tkdv_sir): the
        statistics, m drawn proposal indices and, when asked, their rows of x^
        and the weights of all n proposals."""
        import torch
        dev = torch.device("cuda", self.device)
        K = point.K
        index = torch.empty((max(m, 1),), dtype=torch.int64, device=dev)
        xh = torch.empty((max(m, 1), 2 * K), dtype=torch.float32, device=dev) if rows else None
        w = torch.empty((n,), dtype=torch.float32, device=dev) if weights else None
        st = SirStats()
        _check(lib.tkdv_sir(self._h, C.byref(point), int(proposal), C.byref(plan) if plan is not None else None,
                            int(n), int(m), float(u0), int(precision), _ptr(index), _ptr(xh), _ptr(w),
                            C.byref(st), _stream(stream)), self._h)
        d = st.to_dict()
        d["index"] = index[:m]
        d["xhat"] = xh[:m] if rows else None
        d["weights"] = w
        return d

    def synthesize(self, xhat, precision: int = BF16X3, s3=None, stream=None):
        """s3[r] = sum_j u~_j^3 on the N = 4K grid for rows x^ (n, 2K) float32 on the device."""
        import torch
        assert xhat.dtype == torch.float32 and xhat.is_contiguous() and xhat.dim() == 2
        n, twoK = xhat.shape
        if s3 is None:
            s3 = torch.empty((n,), dtype=torch.float32, device=xhat.device)
        _check(lib.tkdv_synthesize(self._h, twoK // 2, int(precision), _ptr(xhat), int(n), _ptr(s3),
                                   _stream(stream)), self._h)
        return s3

    def eval_proposals(self, point: Point, i0: int, n: int, proposal: int = SIGMA,
                       plan: Plan | None = None, precision: int = BF16X3, stream=None) -> dict:
        """Per-proposal fast-path values and final decisions for indices i0..i0+n-1."""
        import torch
        dev = torch.device("cuda", self.device)
        K = point.K
        out = {
            "xhat": torch.empty((n, 2 * K), dtype=torch.float32, device=dev),
            "t": torch.empty((n,), dtype=torch.float32, device=dev),
            "s3": torch.empty((n,), dtype=torch.float32, device=dev),
            "log_a": torch.empty((n,), dtype=torch.float32, device=dev),
            "log_u": torch.empty((n,), dtype=torch.float32, device=dev),
            "accept": torch.empty((n,), dtype=torch.uint8, device=dev),
        }
        _check(lib.tkdv_eval_proposals(self._h, C.byref(point), int(proposal),
                                       C.byref(plan) if plan is not None else None, int(i0), int(n),
                                       int(precision), _ptr(out["xhat"]), _ptr(out["t"]), _ptr(out["s3"]),
                                       _ptr(out["log_a"]), _ptr(out["log_u"]), _ptr(out["accept"]),
                                       _stream(stream)), self._h)
        return out


def learner_cfg(K: int, hidden: int = 256, eps: float = 0.2, v_amp: float = 0.5, v_scale: float = 0.1,
                temperature: float = 0.05, nll_weight: float = 0.1, lr: float = 3e-3, beta1: float = 0.9,
                beta2: float = 0.999, adam_eps: float = 1e-8, seed: int = 1) -> LearnerCfg:
    return LearnerCfg(int(K), int(hidden), eps, v_amp, v_scale, temperature, nll_weight, lr, beta1, beta2,
                      adam_eps, int(seed))


class Learner:
    """The network of the learned proposal and its training (tkdv_learner_*)."""

    def __init__(self, ctx: Context, cfg: LearnerCfg):
        self._h = C.c_void_p()
        self.cfg = cfg
        self.K = cfg.K
        _check(lib.tkdv_learner_create(ctx._h, C.byref(cfg), C.byref(self._h)))
        self.n_points = 0

    def close(self):
        if self._h:
            lib.tkdv_learner_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_weights(self) -> int:
        return int(lib.tkdv_learner_n_weights(self._h))

    def set_points(self, points: list, sigma_plans: list):
        n = len(points)
        _check(lib.tkdv_learner_set_points(self._h, n, (Point * n)(*points), (Plan * n)(*sigma_plans)))
        self.n_points = n

    def add_rows(self, point: int, xhat, kind: int = 0, stream=None):
        """Rows of one point: a float32 device tensor (n, >= 2K) or a host array (n, 2K)."""
        try:
            import torch
            is_dev = isinstance(xhat, torch.Tensor) and xhat.is_cuda
        except ImportError:
            is_dev = False
        if is_dev:
            assert xhat.dtype == torch.float32 and xhat.dim() == 2 and xhat.stride(1) == 1
            _check(lib.tkdv_learner_add_rows(self._h, int(point), _ptr(xhat), int(xhat.stride(0)),
                                             int(xhat.shape[0]), int(kind), _stream(stream)))
        else:
            x = np.ascontiguousarray(np.asarray(xhat, dtype=np.float64).reshape(-1, 2 * self.K))
            _check(lib.tkdv_learner_add_rows_host(self._h, int(point), x.ctypes.data_as(_PD), x.shape[0],
                                                  int(kind)))

    def add_shifted_rows(self, point: int, xhat, phis, kind: int = 1):
        """Host rows (n, 2K) and their copies translated by each phase in phis
        (the library rotates them on the device); phase 0 keeps a row."""
        x = np.ascontiguousarray(np.asarray(xhat, dtype=np.float64).reshape(-1, 2 * self.K))
        ph = np.ascontiguousarray(np.asarray(phis, dtype=np.float64).reshape(-1))
        _check(lib.tkdv_learner_add_shifted_rows(self._h, int(point), x.ctypes.data_as(_PD), x.shape[0],
                                                 ph.ctypes.data_as(_PD), ph.size, int(kind)))

    def train(self, n_steps: int, stream=None) -> np.ndarray:
        loss = np.zeros(self.n_points)
        _check(lib.tkdv_learner_train(self._h, int(n_steps), loss.ctypes.data_as(_PD), _stream(stream)))
        return loss

    def gradients(self, stream=None):
        """(loss [P], dL/d(log d, V) [P, 5K], dL/dweights [n_weights]) at the current weights."""
        loss = np.zeros(self.n_points)
        gm = np.zeros((self.n_points, 5 * self.K))
        gw = np.zeros(self.n_weights)
        _check(lib.tkdv_learner_gradients(self._h, loss.ctypes.data_as(_PD), gm.ctypes.data_as(_PD),
                                          gw.ctypes.data_as(_PD), _stream(stream)))
        return loss, gm, gw

    def mixture(self, point: Point, sigma_plan: Plan) -> Mixture:
        m = Mixture()
        _check(lib.tkdv_learner_mixture(self._h, C.byref(point), C.byref(sigma_plan), C.byref(m)))
        return m

    def get_weights(self) -> np.ndarray:
        w = np.zeros(self.n_weights)
        _check(lib.tkdv_learner_get_weights(self._h, w.ctypes.data_as(_PD), w.size))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        _check(lib.tkdv_learner_set_weights(self._h, w.ctypes.data_as(_PD), w.size))
