"""Training driver of the learned proposal (the network of ``tkdv_learner``).

Cutting-plane minimax fit of the network's mixtures to a set of training
points, on the GPU:
  1. accepted samples of each point from the paper's sampler (kind-0 rows);
  2. each round: for every point, the network's mixture, its rejection
     constant M_mix = sup f/q_mix (tkdv_plan_mixture_batch: all points at
     once, multi-start L-BFGS on the GPU; or the host's tkdv_plan_mixture),
     and the arg max plus copies of it shifted by fractions of 2 pi/S (the
     target is invariant under every xi-shift, q_mix only under multiples of
     2 pi/S) added as kind-1 rows; then Adam steps on the loss of
     ``tkdv_learner`` (soft maximum of log f/q_mix over the rows plus the
     likelihood term).
The soft maximum pulls down log f/q_mix where it is largest, which is what
sets M_mix and hence the acceptance rate Z/M_mix.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import tkdv as T


@dataclass
class FitResult:
    learner: T.Learner
    points: list
    sigma_plans: list
    history: list = field(default_factory=list)   # per round: per-point log gain, loss, seconds
    best_round: int = -1                           # the round whose weights were kept

    def mixture(self, i: int) -> T.Mixture:
        return self.learner.mixture(self.points[i], self.sigma_plans[i])


def log_M_sigma_normalised(sp: T.Plan) -> float:
    """log sup f/g_Sigma with g_Sigma normalised w.r.t. mu0 (comparable with M_mix)."""
    return sp.log_M - sp.log_norm_g


def plan_mixtures(ctx: T.Context, points: list, sigma_plans: list, mixes: list, starts=None, margin: float = 0.0,
                  seed: int = 0, planner: str = "gpu") -> tuple[list, np.ndarray]:
    """(mixture plans, maximisers [n, 2K]) of many points: on the GPU in one call
    (planner "gpu") or point by point on the host ("host"); starts: None or
    (n, n_user, 2K) caller starts."""
    if planner == "gpu":
        plans, xb = ctx.plan_mixture_batch(points, sigma_plans, mixes, starts=starts, n_starts=16, seed=seed,
                                           margin=margin)
        return plans, xb[:, : 2 * points[0].K] if points else xb
    out, am = [], []
    for i, (pt, sp, mx) in enumerate(zip(points, sigma_plans, mixes)):
        pl, a = T.plan_mixture(pt, sp, mx, starts=None if starts is None else starts[i], margin=margin)
        out.append(pl)
        am.append(a)
    return out, np.array(am)


def fit(ctx: T.Context, points: list, cfg: T.LearnerCfg, samples_per_point: int = 4096, rounds: int = 8,
        steps: int = 150, max_proposals: int = 1 << 32, n_shift_copies: int = 7, margin: float = 0.0,
        precision: int = T.BF16X3, log=None, planner: str = "gpu", nll_samples_per_point: int = 0) -> FitResult:
    """nll_samples_per_point > samples_per_point: that many accepted samples per
    point, the first samples_per_point in both terms of the loss (kind 0), the
    rest in the likelihood term only (kind 2)."""
    sps = [T.plan_point(p, T.SIGMA) for p in points]
    L = T.Learner(ctx, cfg)
    L.set_points(points, sps)
    n_draw = max(samples_per_point, nll_samples_per_point)
    for i, (pt, sp) in enumerate(zip(points, sps)):
        r = ctx.sample(pt, n_draw, proposal=T.SIGMA, plan=sp, mode=T.COUNT_ACCEPTED,
                       max_proposals=max_proposals, precision=precision, capacity=n_draw)
        if r["n_written"] == 0:
            raise RuntimeError(f"point {i}: no accepted sample within {max_proposals} proposals")
        L.add_rows(i, r["xhat"][:samples_per_point], kind=0)
        if r["n_written"] > samples_per_point:
            L.add_rows(i, r["xhat"][samples_per_point:], kind=2)
        del r
    res = FitResult(L, points, sps)
    S = T.MIX_S
    fracs = [2 * math.pi * (q + 1) / ((n_shift_copies + 1) * S) for q in range(n_shift_copies)]
    starts = [[] for _ in points]
    best = (-np.inf, None, -1)
    for rnd in range(rounds + 1):
        t0 = time.time()
        mixes = [L.mixture(pt, sp) for pt, sp in zip(points, sps)]
        st = np.array([s_[-8:] for s_ in starts]) if starts[0] else None
        plans, ams = plan_mixtures(ctx, points, sps, mixes, starts=st, margin=margin, seed=rnd, planner=planner)
        gains = []
        for i, (sp, pl, am) in enumerate(zip(sps, plans, ams)):
            gains.append(log_M_sigma_normalised(sp) - pl.log_M)
            if rnd < rounds:
                L.add_shifted_rows(i, am[None, :], [0.0] + fracs, kind=1)
                starts[i].append(am)
        # the weights of the round with the best mean log M_Sigma/M_mix over the
        # training points (the fit is not monotone in this measure)
        if np.mean(gains) > best[0]:
            best = (float(np.mean(gains)), L.get_weights(), rnd)
        loss = L.train(steps) if rnd < rounds else None
        res.history.append({"round": rnd, "log_gain": gains, "loss": None if loss is None else loss.tolist(),
                            "seconds": time.time() - t0})
        if log:
            g = np.exp(np.array(gains))
            log(f"round {rnd}: M_Sigma/M_mix min {g.min():.2f} median {np.median(g):.2f} max {g.max():.2f}"
                + ("" if loss is None else f", loss {np.mean(loss):.4f}") + f" ({time.time() - t0:.1f}s)")
    L.set_weights(best[1])
    res.best_round = best[2]
    if log:
        log(f"kept the weights of round {best[2]} (mean M_Sigma/M_mix {math.exp(best[0]):.2f})")
    return res


def fit_ensemble(ctx: T.Context, points: list, cfgs: list, log=None, **kw) -> list:
    """fit() from several network initialisations (cfgs differ in their seed):
    the trained networks, all kept (a point's proposal is chosen among them by
    its rejection constant, plan_for_points_ensemble)."""
    out = []
    for cfg in cfgs:
        res = fit(ctx, points, cfg, log=log, **kw)
        if log:
            g = float(np.mean(res.history[res.best_round]["log_gain"]))
            log(f"initialisation seed {cfg.seed}: mean M_Sigma/M_mix {math.exp(g):.2f} over the training points")
        out.append(res)
    return out


def plan_for_points_ensemble(ctx: T.Context, results: list, points: list, margin: float = 0.02,
                             planner: str = "gpu"):
    """Per point, the mixture of the network whose rejection constant M_mix at
    that point is smallest: a point's acceptance is Z/M_mix with Z the same for
    every proposal of the point, so the smallest M gives the highest acceptance
    (plan-time quantities only; every candidate's samples are exact).
    Returns (mixtures, mixture plans, Sigma plans, index of the chosen network)."""
    cands = [plan_for_points(ctx, r, points, margin=margin, planner=planner) for r in results]
    mixes, plans, sps, chosen = [], [], [], []
    for i in range(len(points)):
        e = min(range(len(cands)), key=lambda c: cands[c][1][i].log_M)
        mixes.append(cands[e][0][i])
        plans.append(cands[e][1][i])
        sps.append(cands[e][2][i])
        chosen.append(e)
    return mixes, plans, sps, chosen


def plan_for_points(ctx: T.Context, res_or_learner, points: list, margin: float = 0.02, planner: str = "gpu"):
    """(mixtures, mixture plans, Sigma plans) of the trained network at many points."""
    L = res_or_learner.learner if isinstance(res_or_learner, FitResult) else res_or_learner
    if planner == "gpu":
        sps, _ = ctx.plan_batch(points, T.SIGMA, n_starts=16, seed=1)
    else:
        sps = [T.plan_point(p, T.SIGMA) for p in points]
    mixes = [L.mixture(p, sp) for p, sp in zip(points, sps)]
    plans, _ = plan_mixtures(ctx, points, sps, mixes, margin=margin, planner=planner)
    return mixes, plans, sps


def plan_for(res_or_learner, point: T.Point, margin: float = 0.02, starts=None):
    """(mixture, mixture plan, Sigma plan) of the trained network at any point."""
    L = res_or_learner.learner if isinstance(res_or_learner, FitResult) else res_or_learner
    sp = T.plan_point(point, T.SIGMA)
    mix = L.mixture(point, sp)
    pl, _ = T.plan_mixture(point, sp, mix, starts=starts, margin=margin)
    return mix, pl, sp
