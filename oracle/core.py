"""ctypes bindings of the C FP64 oracle (``tkdv_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The shared library is built by ``build_oracle()`` (gcc, -O2, OpenMP); it is
compiled on first use when it is missing.  The environment variable
``TKDV_ORACLE_LIB`` points the bindings at another build of the same source
(used by the mutation test, which plants mistakes in a copy of the source).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tkdv_oracle.c")
_LIB = os.path.join(_HERE, "libtkdv_oracle.so")

NBINS = 64


def build_oracle(extra_flags: list[str] | None = None, out: str | None = None) -> str:
    """Compile the C oracle with gcc; returns the path of the shared library."""
    out = out or _LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
           "-o", out, _SRC, "-lm"] + list(extra_flags or [])
    subprocess.run(cmd, check=True)
    return out


def _load(path: str | None = None) -> C.CDLL:
    path = path or os.environ.get("TKDV_ORACLE_LIB") or _LIB
    if not os.path.exists(path):
        build_oracle(out=path)
    return C.CDLL(path)


class _Point(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("N", C.c_int32), ("proposal", C.c_int32), ("point_id", C.c_uint32),
        ("E0", C.c_double), ("beta_p", C.c_double), ("c32", C.c_double),
        ("alpha_star", C.c_double), ("log_M", C.c_double), ("seed", C.c_uint64),
    ]


class _Stats(C.Structure):
    _fields_ = [
        ("n_proposed", C.c_uint64), ("n_accepted", C.c_uint64), ("n_written", C.c_uint64),
        ("n_violations", C.c_uint64), ("n_exceed", C.c_uint64), ("n_grid", C.c_uint64),
        ("max_log_a", C.c_double),
        ("S1", C.c_double), ("S2", C.c_double), ("S3", C.c_double), ("S4", C.c_double),
        ("skewness", C.c_double), ("kurtosis", C.c_double), ("p_exceed", C.c_double),
        ("hist_lo", C.c_double), ("hist_hi", C.c_double),
        ("hist", C.c_uint64 * NBINS),
        ("n_exceed4", C.c_uint64), ("n_max4", C.c_uint64), ("peak_u", C.c_double), ("peak_index", C.c_uint64),
    ]


MIX_S, MIX_R = 32, 2


class _Mixture(C.Structure):
    _fields_ = [("K", C.c_int32), ("pad", C.c_int32), ("eps", C.c_double),
                ("logd", C.c_double * 128), ("V", (C.c_double * MIX_R) * 256)]


def make_mixture(K: int, eps: float, logd, V) -> _Mixture:
    """Base component L0 = D + V V^T: logd [K], V [2K, 2]."""
    m = _Mixture()
    m.K, m.eps = K, eps
    logd = np.asarray(logd, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    for k in range(K):
        m.logd[k] = logd[k]
    for c in range(2 * K):
        for q in range(MIX_R):
            m.V[c][q] = V[c, q]
    return m


@dataclass
class OracleStats:
    n_proposed: int
    n_accepted: int
    n_written: int
    n_violations: int
    n_exceed: int
    n_grid: int
    max_log_a: float
    S1: float
    S2: float
    S3: float
    S4: float
    skewness: float
    kurtosis: float
    p_exceed: float
    hist_lo: float
    hist_hi: float
    hist: np.ndarray
    n_exceed4: int = 0      # grid values above 4 sigma = 4 sqrt(E0/pi)
    n_max4: int = 0         # samples whose largest grid value is above 4 sigma
    peak_u: float = -math.inf   # largest grid value over the samples
    peak_index: int = 2**64 - 1  # index of the sample attaining it (lowest among equal)

    @classmethod
    def _from(cls, s: _Stats) -> "OracleStats":
        return cls(s.n_proposed, s.n_accepted, s.n_written, s.n_violations, s.n_exceed,
                   s.n_grid, s.max_log_a, s.S1, s.S2, s.S3, s.S4, s.skewness, s.kurtosis,
                   s.p_exceed, s.hist_lo, s.hist_hi, np.array(s.hist[:], dtype=np.uint64),
                   s.n_exceed4, s.n_max4, s.peak_u, s.peak_index)

    @property
    def acceptance(self) -> float:
        return self.n_accepted / self.n_proposed if self.n_proposed else float("nan")


_D = C.c_double
_PD = C.POINTER(C.c_double)
_PU32 = C.POINTER(C.c_uint32)

lib = _load()
lib.orc_philox4x32_10.argtypes = [_PU32, _PU32, _PU32]
lib.orc_proposal_words.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _PU32]
lib.orc_uniform.argtypes = [C.c_uint32]
lib.orc_uniform.restype = _D
lib.orc_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_int, _PD, _PD, _PD]
lib.orc_sigma2.argtypes = [C.c_int, _D, _D, C.c_int]
lib.orc_sigma2.restype = _D
lib.orc_F_alpha.argtypes = [C.c_int, _D, _D]
lib.orc_F_alpha.restype = _D
lib.orc_t.argtypes = [C.c_int, _PD]
lib.orc_t.restype = _D
lib.orc_H2.argtypes = [C.c_int, _D, _PD]
lib.orc_H2.restype = _D
lib.orc_H3_triad.argtypes = [C.c_int, _D, _PD]
lib.orc_H3_triad.restype = _D
lib.orc_H3_quad.argtypes = [C.c_int, _D, C.c_int, _PD]
lib.orc_H3_quad.restype = _D
lib.orc_grid.argtypes = [C.c_int, _D, C.c_int, _PD, _PD]
lib.orc_log_ratio.argtypes = [C.c_int, _D, _D, _D, _D, C.c_int, _PD]
lib.orc_log_ratio.restype = _D
lib.orc_log_ratio_unnorm.argtypes = [C.c_int, _D, _D, _D, _D, C.c_int, _PD]
lib.orc_log_ratio_unnorm.restype = _D
lib.orc_proposal.argtypes = [C.POINTER(_Point), C.c_uint64, _PD, _PD]
lib.orc_proposal.restype = _D
lib.orc_sample.argtypes = [C.POINTER(_Point), C.c_uint64, C.c_uint64, C.POINTER(C.c_uint8),
                           _PD, _PD, _PD, C.POINTER(C.c_uint64), C.c_uint64,
                           C.POINTER(_Stats), C.c_int]
lib.orc_sample.restype = C.c_uint64
lib.orc_sample_until.argtypes = [C.POINTER(_Point), C.c_uint64, C.c_uint64, _PD,
                                 C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(_Stats), C.c_int]
lib.orc_sample_until.restype = C.c_uint64
lib.orc_stats_of.argtypes = [C.c_int, C.c_int, _D, _PD, C.c_uint64, C.POINTER(_Stats)]
lib.orc_eval_batch.argtypes = [C.POINTER(_Point), C.c_uint64, C.c_uint64, _PD, _PD, _PD, _PD, _PD, _PD, C.c_int]
lib.orc_shift.argtypes = [C.c_int, _D, _PD, _PD]
lib.orc_sir.argtypes = [C.POINTER(_Point), C.c_uint64, C.c_uint64, C.c_uint64, _D, _PD,
                        C.POINTER(C.c_uint64), _PD, C.c_int]
lib.orc_mix_log_q.argtypes = [C.POINTER(_Point), C.POINTER(_Mixture), _PD, _PD, _PD]
lib.orc_mix_draw.argtypes = [C.POINTER(_Point), C.POINTER(_Mixture), C.c_uint64, _PD, _PD]
lib.orc_mix_draw.restype = C.c_int
lib.orc_mix_proposal.argtypes = [C.POINTER(_Point), C.POINTER(_Mixture), C.c_uint64, _PD, _PD]
lib.orc_mix_proposal.restype = _D
lib.orc_mix_sample.argtypes = [C.POINTER(_Point), C.POINTER(_Mixture), C.c_uint64, C.c_uint64,
                               C.POINTER(C.c_uint8), _PD, _PD, _PD, C.POINTER(C.c_uint64), C.c_uint64, C.c_int]
lib.orc_mix_sample.restype = C.c_uint64
lib.orc_mix_threshold.argtypes = [C.POINTER(_Mixture)]
lib.orc_mix_threshold.restype = C.c_uint64
lib.orc_mix_eps.argtypes = [C.POINTER(_Mixture)]
lib.orc_mix_eps.restype = _D
lib.orc_hist_bin.argtypes = [_D, _D]
lib.orc_hist_bin.restype = C.c_int
lib.orc_max_threads.restype = C.c_int


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_PD)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(c.ctypes.data_as(_PU32), k.ctypes.data_as(_PU32), out.ctypes.data_as(_PU32))
    return out


def proposal_words(seed: int, i: int, point_id: int, K: int, tag: int = 0) -> np.ndarray:
    nw = 2 * K + 2
    out = np.zeros(nw, dtype=np.uint32)
    lib.orc_proposal_words(seed, i, point_id, tag, nw, out.ctypes.data_as(_PU32))
    return out


def uniform_of_word(w: int) -> float:
    return lib.orc_uniform(int(w))


def normals(seed: int, i: int, point_id: int, K: int):
    """(z[2K], U_accept, U_mix) of proposal i."""
    z = np.zeros(2 * K)
    ua = C.c_double()
    um = C.c_double()
    lib.orc_normals(seed, i, point_id, K, _dp(z), C.byref(ua), C.byref(um))
    return z, ua.value, um.value


def t_of(xh) -> float:
    x = _f64(xh)
    return lib.orc_t(x.size // 2, _dp(x))


def H2(xh, E0: float) -> float:
    x = _f64(xh)
    return lib.orc_H2(x.size // 2, E0, _dp(x))


def H3_triad(xh, E0: float) -> float:
    x = _f64(xh)
    return lib.orc_H3_triad(x.size // 2, E0, _dp(x))


def H3_quad(xh, E0: float, N: int) -> float:
    x = _f64(xh)
    return lib.orc_H3_quad(x.size // 2, E0, N, _dp(x))


def grid(xh, E0: float, N: int) -> np.ndarray:
    x = _f64(xh)
    u = np.zeros(N)
    lib.orc_grid(x.size // 2, E0, N, _dp(x), _dp(u))
    return u


def extremes(xhat, E0: float, N: int, top_k: int, threshold: float) -> dict:
    """Largest surface displacement of each row (Sec. V, individual wave fields):
    u on the N-point grid xi_j = -pi + 2 pi j/N (``grid``), its maximum and
    the first grid index attaining it; the top_k rows by maximum (descending,
    ties by lower row index); the number of rows whose maximum exceeds
    `threshold`."""
    x = np.asarray(xhat, dtype=np.float64)
    n = x.shape[0]
    um = np.empty(n)
    jm = np.empty(n, dtype=np.int64)
    for r in range(n):
        u = grid(x[r], E0, N)
        jm[r] = int(np.argmax(u))
        um[r] = u[jm[r]]
    order = np.lexsort((np.arange(n), -um))[:top_k]
    return {"umax": um, "jmax": jm, "rows": order, "n_exceed": int(np.sum(um > threshold))}


def log_ratio(xh, E0, beta_p, c32, alpha, proposal_kind: int, normalise_input=False) -> float:
    """log f/g (proposal_kind 1) or log f (0), unnormalised, at x^ (or y/|y|)."""
    x = _f64(xh)
    fn = lib.orc_log_ratio_unnorm if normalise_input else lib.orc_log_ratio
    return fn(x.size // 2, E0, beta_p, c32, alpha, proposal_kind, _dp(x))


def F_alpha(K: int, beta_p: float, alpha: float) -> float:
    return lib.orc_F_alpha(K, beta_p, alpha)


def _point(K, N, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed) -> _Point:
    return _Point(K, N, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)


def proposal(K, E0, beta_p, c32, proposal_kind, alpha_star, log_M, seed, point_id, i, N=None):
    """(x^, log a, log U) of proposal i."""
    p = _point(K, N or 4 * K, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)
    xh = np.zeros(2 * K)
    lu = C.c_double()
    la = lib.orc_proposal(C.byref(p), i, _dp(xh), C.byref(lu))
    return xh, la, lu.value


def sample(K, E0, beta_p, c32, proposal_kind, alpha_star, log_M, seed, point_id, n,
           N, i0=0, cap=0, want_log=False, nthreads=0):
    """Run the sampler over proposal indices [i0, i0+n).

    Returns dict with accept (uint8[n]), optional log_a/log_u, xhat [min(cap,
    n_acc), 2K], index, stats.
    """
    p = _point(K, N, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)
    acc = np.zeros(n, dtype=np.uint8)
    la = np.zeros(n) if want_log else None
    lu = np.zeros(n) if want_log else None
    xo = np.zeros((max(cap, 1), 2 * K))
    io = np.zeros(max(cap, 1), dtype=np.uint64)
    st = _Stats()
    lib.orc_sample(C.byref(p), i0, n, acc.ctypes.data_as(C.POINTER(C.c_uint8)),
                   _dp(la) if la is not None else None, _dp(lu) if lu is not None else None,
                   _dp(xo), io.ctypes.data_as(C.POINTER(C.c_uint64)), cap, C.byref(st), nthreads)
    s = OracleStats._from(st)
    nw = s.n_written
    return {"accept": acc, "log_a": la, "log_u": lu, "xhat": xo[:nw], "index": io[:nw], "stats": s}


def sample_until(K, E0, beta_p, c32, proposal_kind, alpha_star, log_M, seed, point_id,
                 n_target, max_proposals, N, cap=None, nthreads=0):
    """Accepted-count mode: the first n_target accepted samples by index."""
    cap = n_target if cap is None else cap
    p = _point(K, N, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)
    xo = np.zeros((max(cap, 1), 2 * K))
    io = np.zeros(max(cap, 1), dtype=np.uint64)
    st = _Stats()
    lib.orc_sample_until(C.byref(p), n_target, max_proposals, _dp(xo),
                         io.ctypes.data_as(C.POINTER(C.c_uint64)), cap, C.byref(st), nthreads)
    s = OracleStats._from(st)
    return {"xhat": xo[:s.n_written], "index": io[:s.n_written], "stats": s}


def eval_batch(K, E0, beta_p, c32, proposal_kind, alpha_star, log_M, seed, point_id, i0, n, N,
               grid=True, nthreads=0) -> dict:
    """Per-proposal H2, H3 (double sum), grid sums S3/S3abs of the unscaled field
    (when grid), log a and log U for indices i0..i0+n-1."""
    p = _point(K, N, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)
    out = {k: np.zeros(n) for k in ("H2", "H3", "log_a", "log_u")}
    if grid:
        out["S3"], out["S3abs"] = np.zeros(n), np.zeros(n)
    g = (lambda k: _dp(out[k]) if k in out else None)
    lib.orc_eval_batch(C.byref(p), i0, n, g("H2"), g("H3"), g("S3"), g("S3abs"), g("log_a"), g("log_u"),
                       nthreads)
    return out


def sir(K, E0, beta_p, c32, proposal_kind, alpha_star, log_M, seed, point_id, n, m, u0, i0=0, N=None,
        nthreads=0) -> dict:
    """Sampling-importance resampling over proposal indices i0..i0+n-1 with the
    paper's proposal (orc_sir): weights w_i = f/(M g), their sums, the
    self-normalised grid moments and m systematic draws with offset u0."""
    p = _point(K, N or 4 * K, proposal_kind, point_id, E0, beta_p, c32, alpha_star, log_M, seed)
    w = np.zeros(max(n, 1))
    idx = np.zeros(max(m, 1), dtype=np.uint64)
    sums = np.zeros(8)
    lib.orc_sir(C.byref(p), i0, n, m, float(u0), _dp(w), idx.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(sums),
                nthreads)
    W, W2 = sums[0], sums[1]
    m2 = sums[4]
    return {"weights": w[:n], "index": idx[:m], "W": W, "W2": W2, "ess": W * W / W2 if W2 > 0 else 0.0,
            "max_w": sums[2], "moments": sums[3:7].copy(), "n_over_one": int(sums[7]),
            "skewness": sums[5] / m2 ** 1.5 if m2 > 0 else 0.0, "kurtosis": sums[6] / m2 ** 2 if m2 > 0 else 0.0}


def shift(x, phi: float) -> np.ndarray:
    """Coefficients of u(xi + phi): mode k rotated by the angle k phi."""
    x = _f64(x)
    out = np.zeros_like(x)
    lib.orc_shift(x.size // 2, phi, _dp(x), _dp(out))
    return out


def mix_log_q(K, E0, beta_p, c32, alpha_star, mixture, xhat):
    """(log q_net, log q_mix) at x^ (normalised densities w.r.t. mu0)."""
    p = _point(K, 4 * K, 1, 0, E0, beta_p, c32, alpha_star, 0.0, 0)
    x = _f64(xhat)
    a, b = C.c_double(), C.c_double()
    lib.orc_mix_log_q(C.byref(p), C.byref(mixture), _dp(x), C.byref(a), C.byref(b))
    return a.value, b.value


def mix_draw(K, E0, beta_p, c32, alpha_star, mixture, seed, point_id, i):
    """(x^, component or -1, log U) of mixture proposal i."""
    p = _point(K, 4 * K, 1, point_id, E0, beta_p, c32, alpha_star, 0.0, seed)
    xh = np.zeros(2 * K)
    lu = C.c_double()
    comp = lib.orc_mix_draw(C.byref(p), C.byref(mixture), i, _dp(xh), C.byref(lu))
    return xh, comp, lu.value


def mix_proposal(K, E0, beta_p, c32, alpha_star, log_M_mix, mixture, seed, point_id, i):
    """(x^, log a, log U) of mixture proposal i (log a with log M_mix)."""
    p = _point(K, 4 * K, 1, point_id, E0, beta_p, c32, alpha_star, log_M_mix, seed)
    xh = np.zeros(2 * K)
    lu = C.c_double()
    la = lib.orc_mix_proposal(C.byref(p), C.byref(mixture), i, _dp(xh), C.byref(lu))
    return xh, la, lu.value


def mix_sample(K, E0, beta_p, c32, alpha_star, log_M_mix, mixture, seed, point_id, n, i0=0,
               cap=0, want_log=False, nthreads=0):
    """Rejection sampler with the mixture proposal over indices [i0, i0+n)."""
    p = _point(K, 4 * K, 1, point_id, E0, beta_p, c32, alpha_star, log_M_mix, seed)
    acc = np.zeros(n, dtype=np.uint8)
    la = np.zeros(n) if want_log else None
    lu = np.zeros(n) if want_log else None
    xo = np.zeros((max(cap, 1), 2 * K))
    io = np.zeros(max(cap, 1), dtype=np.uint64)
    nacc = lib.orc_mix_sample(C.byref(p), C.byref(mixture), i0, n, acc.ctypes.data_as(C.POINTER(C.c_uint8)),
                              _dp(la) if la is not None else None, _dp(lu) if lu is not None else None,
                              _dp(xo), io.ctypes.data_as(C.POINTER(C.c_uint64)), cap, nthreads)
    nw = min(nacc, cap)
    return {"accept": acc, "log_a": la, "log_u": lu, "xhat": xo[:nw], "index": io[:nw], "n_accepted": nacc}


def mix_eps(mixture) -> float:
    """Weight of g_Sigma the mixture realises: E 2^-32, E = S floor(eps 2^32/S)."""
    return lib.orc_mix_eps(C.byref(mixture))


def mix_threshold(mixture) -> int:
    return int(lib.orc_mix_threshold(C.byref(mixture)))


def stats_of(xhat, E0: float, N: int) -> OracleStats:
    x = _f64(xhat)
    if x.ndim == 1:
        x = x[None, :]
    K = x.shape[1] // 2
    st = _Stats()
    lib.orc_stats_of(K, N, E0, _dp(x), x.shape[0], C.byref(st))
    return OracleStats._from(st)


def hist_bin(u0: float, u_max: float) -> int:
    return lib.orc_hist_bin(u0, u_max)


def max_threads() -> int:
    return lib.orc_max_threads()
