"""Sampling-importance resampling on the GPU (tkdv_sir) against the oracle.

* Weights: |log w_gpu - log w_oracle| <= tau/2, the fast path's error bound
  (the decision window of the rejection step, tkdv_decision_window); hence W,
  W2 and the ESS within that relative error.
* Moments: the weighted grid mean is 0 and the mean square E0/pi (Parseval);
  m3, m4, skewness and kurtosis within the weight error of the oracle's.
* Draws: equal to the oracle's except where the draw's position (u0 + r) W/m
  lies within the accumulated weight error of a cumulative boundary; the rows
  of x^ of the drawn proposals equal the oracle's proposals.
* Equal weights (beta' = 0, uniform proposal, log M = 0): draw r is proposal
  floor((u0 + r) n/m) exactly.
* Ragged n, m = 0, n = 1, determinism, argument errors.
* K = 128 (the quarter-period kernels): the same checks; S4 there is formed on
  the grid offset by half a step and carried to the grid xi_j by the closed
  form of the difference, which the m4 and kurtosis checks cover.
"""
import math
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_16952_amd import tkdv
    return tkdv


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


CASES = [  # K, E0, beta', C3/C2, proposal, n, m, u0, precision name
    (8, 1.0, 40.0, 20.0, 1, 200_003, 5000, 0.37, "bf16x3"),
    (8, 1.0, 40.0, 20.0, 1, 200_003, 5000, 0.37, "fp32"),
    (16, 2.0, 40.0, 60.0, 1, 100_001, 3000, 0.0, "bf16x3"),
    (32, 1.0, 40.0, 75.0, 1, 60_000, 2000, 0.91, "bf16x3"),
    (16, 1.0, 40.0, 30.0, 0, 150_000, 1000, 0.5, "fp32"),
    (64, 1.0, 40.0, 150.0, 1, 20_000, 700, 0.2, "bf16x3"),
    (128, 1.0, 40.0, 1000.0, 1, 12_011, 600, 0.45, "bf16x3"),  # quarter-period weights and rows
    (128, 1.5, 40.0, 750.0, 1, 8_003, 400, 0.05, "fp32"),
]


@pytest.mark.parametrize("K,E0,bp,c,prop,n,m,u0,prec", CASES)
def test_sir_against_oracle(T, ctx, K, E0, bp, c, prop, n, m, u0, prec):
    P = T.PRECISIONS[prec]
    pt = T.make_point(K, E0, bp, c, seed=4, point_id=2)
    pl = T.plan_point(pt, prop)
    tau = T.decision_window(pt, prop, P)
    g = ctx.sir(pt, n, m, u0, proposal=prop, plan=pl, precision=P, rows=True, weights=True)
    o = oracle.sir(K, E0, bp, c, prop, pl.alpha_star, pl.log_M, 4, 2, n, m, u0)
    wg = g["weights"].cpu().numpy().astype(np.float64)
    wo = o["weights"]
    ok = wo > 1e-30
    lerr = np.max(np.abs(np.log(wg[ok]) - np.log(wo[ok])))
    say(f"K={K} {prec} prop={prop}: W gpu {g['W']:.10g} oracle {o['W']:.10g}; ESS {g['ess']:.6g} / {o['ess']:.6g}; "
        f"max |dlog w| {lerr:.2e} (tau/2 {tau / 2:.2e}); skew {g['skewness']:.5f} / {o['skewness']:.5f}")
    assert lerr <= tau / 2
    rel = tau / 2 + 1e-12
    assert abs(g["W"] / o["W"] - 1) <= rel
    assert abs(g["W2"] / o["W2"] - 1) <= 2 * rel
    assert abs(g["ess"] / o["ess"] - 1) <= 4 * rel
    assert abs(g["max_w"] / o["max_w"] - 1) <= rel
    assert g["n_over_one"] == o["n_over_one"] == 0
    # moments: Parseval fixes the first two; the rest follow the weights
    assert abs(g["mean"]) < 1e-5 * math.sqrt(E0)
    assert abs(g["m2"] / (E0 / math.pi) - 1) < 3e-5
    mo = o["moments"]
    assert abs(g["m3"] - mo[2]) <= (2 * rel + 3e-5) * mo[3] ** 0.75
    assert abs(g["m4"] / mo[3] - 1) <= 2 * rel + 3e-5
    # draws
    ig = g["index"].cpu().numpy().astype(np.int64)
    io = o["index"].astype(np.int64)
    assert len(ig) == m and np.all(np.diff(ig) >= 0) and ig.min() >= 0 and ig.max() < n
    C = np.cumsum(wo)
    bad = np.nonzero(ig != io)[0]
    for r in bad:
        pos = (u0 + r) * o["W"] / m
        lo, hi = sorted((ig[r], io[r]))
        # a boundary between the two choices lies within the accumulated error
        gap = np.min(np.abs(C[lo:hi] - pos))
        assert gap <= tau * o["W"], f"draw {r}: {ig[r]} vs {io[r]}, nearest boundary {gap:.3e}"
    say(f"   {len(bad)} of {m} draws differ (all at boundaries within the weight error)")
    assert len(bad) <= max(2, m // 100)
    # rows of the drawn proposals
    xg = g["xhat"].cpu().numpy().astype(np.float64)
    for r in np.random.default_rng(1).integers(0, m, 40):
        x, _, _ = oracle.proposal(K, E0, bp, c, prop, pl.alpha_star, pl.log_M, 4, 2, int(ig[r]))
        assert np.linalg.norm(xg[r] - x) < 2e-6


def test_equal_weights_closed_form(T, ctx):
    K, n, m, u0 = 16, 100_000, 3_331, 0.3141592653589793
    pt = T.make_point(K, 1.0, 0.0, 0.0, seed=1, point_id=0)
    pl = T.plan_point(pt, T.UNIFORM)
    assert pl.log_M == 0.0
    pos = (u0 + np.arange(m)) * n / m
    assert np.min(np.abs(pos - np.round(pos))) > 1e-6   # no draw sits on a boundary
    g = ctx.sir(pt, n, m, u0, proposal=T.UNIFORM, plan=pl, precision=T.FP32)
    assert g["W"] == n and g["W2"] == n and g["max_w"] == 1.0
    assert g["index"].cpu().numpy().tolist() == [math.floor(p) for p in pos]
    assert g["kurtosis"] == pytest.approx(3 * K / (K + 1), abs=0.02)


def test_edges_determinism_and_errors(T, ctx):
    K = 8
    pt = T.make_point(K, 1.0, 40.0, 20.0, seed=0, point_id=0)
    pl = T.plan_point(pt, T.SIGMA)
    a = ctx.sir(pt, 50_001, 997, 0.6, plan=pl)
    b = ctx.sir(pt, 50_001, 997, 0.6, plan=pl)
    assert a["W"] == b["W"] and a["ess"] == b["ess"]
    assert np.array_equal(a["index"].cpu().numpy(), b["index"].cpu().numpy())
    s0 = ctx.sir(pt, 50_001, 0, 0.6, plan=pl)                 # statistics only
    assert s0["W"] == a["W"] and len(s0["index"]) == 0
    one = ctx.sir(pt, 1, 5, 0.0, plan=pl)                    # a single proposal takes every draw
    assert one["index"].cpu().numpy().tolist() == [0] * 5
    with pytest.raises(T.TkdvError):
        ctx.sir(pt, 1000, 10, 0.5, plan=pl, precision=T.BF16)
    with pytest.raises(T.TkdvError):
        ctx.sir(pt, 1000, 10, 1.0, plan=pl)
    with pytest.raises(T.TkdvError):
        ctx.sir(pt, 0, 10, 0.5, plan=pl)
    with pytest.raises(T.TkdvError):
        ctx.sir(pt, 1000, 10, 0.5, proposal=T.UNIFORM, plan=pl)   # plan of the other proposal
