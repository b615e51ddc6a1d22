"""Per-point precompute of the rejection algorithm (step 1 of Sec. IV.B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``alpha_star``: the root of F(alpha) = 1 - (alpha/K) sum_k 1/(1 + alpha beta' k^2/K^3)
  (Sec. III.A), by scipy's Brent root finder on a bracket found by doubling.
  F(0) = 1 and F is strictly decreasing, with F(inf) = 1 - (K^2/beta') sum 1/k^2,
  so a root exists iff 0 <= beta' < K^2 sum_{k<=K} 1/k^2 (reading adopted for
  the paper's "selected as the root").
* ``sigma2``: sigma_k^2 = 1/(1 + alpha* beta' k^2/K^3) (Sec. III.A).
* ``log_M``: log of M = sup over the sphere of f/g (Sec. IV.A), found as the
  paper describes, by Nelder-Mead started at the zero-mean Dirichlet kernel
  u^_k = sqrt(E0/(2 pi K)); additional starts (all energy in mode 1, seeded
  random directions) and Nelder-Mead restarts from the incumbent guard against
  a local maximum.  The function maximised is y -> log(f/g)(y/|y|) on R^{2K}.
  For the linear case C3/C2 = 0 the ratio depends on t = sum k^2 s_k only, and
  M has the closed form used by ``log_M_linear``.

The result of the optimisation is a lower bound on the true supremum; its
agreement with the closed form (C3/C2 = 0) and with the HIP library's own
search is checked by the tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import optimize

from . import core

UNIFORM, SIGMA = 0, 1


class NoAlphaRoot(ValueError):
    pass


def alpha_root_exists(K: int, beta_p: float) -> bool:
    return 0.0 <= beta_p < K * K * sum(1.0 / (k * k) for k in range(1, K + 1))


def alpha_star(K: int, beta_p: float) -> float:
    if beta_p < 0:
        raise ValueError("beta' must be >= 0")
    if beta_p == 0.0:
        return 1.0
    if not alpha_root_exists(K, beta_p):
        raise NoAlphaRoot(f"F has no root for K={K}, beta'={beta_p}")
    hi = 1.0
    while core.F_alpha(K, beta_p, hi) > 0.0:
        hi *= 2.0
        if hi > 1e300:
            raise NoAlphaRoot("bracket search failed")
    return optimize.brentq(lambda a: core.F_alpha(K, beta_p, a), 0.0, hi,
                           xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)


def sigma2(K: int, beta_p: float, alpha: float) -> np.ndarray:
    k = np.arange(1, K + 1, dtype=np.float64)
    return 1.0 / (1.0 + alpha * beta_p * k * k / float(K) ** 3)


def log_M_linear(K: int, beta_p: float, alpha: float, proposal: int) -> float:
    """Closed-form log M for C3/C2 = 0.

    Sigma proposal: f/g = h(t) = exp(-beta' t/K^2) (1 + alpha beta' t/K^3)^K, log h
    concave in t, stationary at t* = K^3 (alpha - 1)/(alpha beta'), clamped to the
    attainable range [1, K^2].  Uniform proposal: f = exp(-beta' t/K^2), largest at t = 1.
    """
    if proposal == UNIFORM:
        return -beta_p / K**2
    if beta_p == 0.0:
        return 0.0
    ts = K**3 * (alpha - 1.0) / (alpha * beta_p)
    ts = min(max(ts, 1.0), float(K * K))
    return -beta_p * ts / K**2 + K * math.log1p(alpha * beta_p * ts / K**3)


def dirichlet_direction(K: int) -> np.ndarray:
    """Zero-mean Dirichlet kernel u^_k = sqrt(E0/(2 pi K)) as a point of the sphere."""
    y = np.zeros(2 * K)
    y[:K] = 1.0 / math.sqrt(K)
    return y


@dataclass
class OraclePlan:
    K: int
    E0: float
    beta_p: float
    c32: float
    proposal: int
    alpha_star: float
    sigma2: np.ndarray
    log_M: float
    argmax: np.ndarray = field(repr=False)
    closed_form: bool = False


def _maximise(fun, y0: np.ndarray, max_restarts: int = 12) -> tuple[float, np.ndarray]:
    """Nelder-Mead (adaptive coefficients) on -fun, restarted from the incumbent.

    The ratio is invariant under shifts in xi, so its maximiser is a curve and
    the simplex need not shrink along it; termination therefore uses a loose x
    tolerance and a tight value tolerance, and restarts continue until a
    restart gains less than 1e-14.
    """
    best_y = y0 / np.linalg.norm(y0)
    best = fun(best_y)
    for _ in range(max_restarts):
        res = optimize.minimize(lambda y: -fun(y), best_y, method="Nelder-Mead",
                                options=dict(adaptive=True, xatol=1e-6, fatol=1e-13,
                                             maxiter=400_000, maxfev=400_000))
        y = res.x / np.linalg.norm(res.x)
        val = fun(y)
        improved = val > best + 1e-14
        if val > best:
            best, best_y = val, y
        if not improved:
            break
    return best, best_y


def log_M(K: int, E0: float, beta_p: float, c32: float, proposal: int, alpha: float,
          n_random: int = 2, seed: int = 12345) -> tuple[float, np.ndarray]:
    """log M = log sup f/g (Sigma) or log sup f (uniform), by multi-start Nelder-Mead."""
    def fun(y):
        return core.log_ratio(y, E0, beta_p, c32, alpha, proposal, normalise_input=True)

    starts = [dirichlet_direction(K)]
    e1 = np.zeros(2 * K)
    e1[0] = 1.0
    starts.append(e1)
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        starts.append(rng.standard_normal(2 * K))
    best, best_y = -np.inf, None
    for y0 in starts:
        v, y = _maximise(fun, y0)
        if v > best:
            best, best_y = v, y
    return best, best_y


def plan_point(K: int, E0: float, beta_p: float, c32: float, proposal: int = SIGMA,
               n_random: int = 2, seed: int = 12345) -> OraclePlan:
    a = alpha_star(K, beta_p) if proposal == SIGMA else 1.0
    s2 = sigma2(K, beta_p, a) if proposal == SIGMA else np.ones(K)
    if c32 == 0.0:
        lm = log_M_linear(K, beta_p, a, proposal)
        return OraclePlan(K, E0, beta_p, c32, proposal, a, s2, lm, np.zeros(2 * K), True)
    lm, y = log_M(K, E0, beta_p, c32, proposal, a, n_random=n_random, seed=seed)
    return OraclePlan(K, E0, beta_p, c32, proposal, a, s2, lm, y, False)
