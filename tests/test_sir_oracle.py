"""Pins of the oracle's sampling-importance resampling (oracle.sir), no GPU.

* Equal weights (beta' = 0, uniform proposal, log M = 0: f = g): W = ESS = n
  and draw r is proposal floor((u0 + r) n/m) exactly; the grid kurtosis is the
  uniform-sphere law's 3K/(K+1) within sampling error.
* For any weights, the self-normalised moments obey Parseval: the grid mean
  of u is 0 and the grid mean of u^2 is E0/pi for every sample (N > 2K).
* The weights are exp(log a) of the rejection sampler's own decisions.
* Systematic resampling gives proposal i either floor(m w_i/W) or
  ceil(m w_i/W) copies, in increasing proposal order.
* The SIR estimate of the skewness agrees with the rejection sampler's
  (K = 8, beta' = 40, C3/C2 = 20, skewness about 0.55) within sampling error.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import plan as OP


def test_equal_weights_closed_forms():
    K, n, m, u0 = 8, 20000, 777, 0.3
    r = oracle.sir(K, 1.0, 0.0, 20.0, 0, 1.0, 0.0, 3, 0, n, m, u0)
    assert r["W"] == n and r["ess"] == pytest.approx(n, rel=1e-14)
    assert r["index"].tolist() == [math.floor((u0 + j) * n / m) for j in range(m)]
    assert r["kurtosis"] == pytest.approx(3 * K / (K + 1), abs=0.03)
    assert abs(r["skewness"]) < 0.03


@pytest.mark.parametrize("K,E0,bp,c,n", [(8, 1.0, 40.0, 20.0, 5000), (16, 2.0, 40.0, 60.0, 5000),
                                         (128, 1.5, 40.0, 750.0, 400)])
def test_parseval_moments_for_any_weights(K, E0, bp, c, n):
    if K == 128:  # the plan only sets the weights' scale; any log M keeps Parseval
        alpha, log_M = 1.0, 0.0
    else:
        p = OP.plan_point(K, E0, bp, c, proposal=1, n_random=0)
        alpha, log_M = p.alpha_star, p.log_M
    r = oracle.sir(K, E0, bp, c, 1, alpha, log_M, 1, 2, n, 10, 0.5)
    assert abs(r["moments"][0]) < 1e-12
    assert r["moments"][1] == pytest.approx(E0 / math.pi, rel=1e-12)


def test_weights_are_the_rejection_probabilities():
    K, bp, c = 8, 40.0, 20.0
    p = OP.plan_point(K, 1.0, bp, c, proposal=1, n_random=0)
    r = oracle.sir(K, 1.0, bp, c, 1, p.alpha_star, p.log_M, 0, 0, 3000, 5, 0.5, i0=100)
    e = oracle.eval_batch(K, 1.0, bp, c, 1, p.alpha_star, p.log_M, 0, 0, 100, 3000, 4 * K, grid=False)
    assert np.allclose(r["weights"], np.exp(e["log_a"]), rtol=1e-15, atol=0)


def test_systematic_resampling_counts():
    K, bp, c, n, m = 8, 40.0, 20.0, 5000, 2000
    p = OP.plan_point(K, 1.0, bp, c, proposal=1, n_random=0)
    r = oracle.sir(K, 1.0, bp, c, 1, p.alpha_star, p.log_M, 5, 0, n, m, 0.71)
    idx = r["index"].astype(np.int64)
    assert np.all(np.diff(idx) >= 0) and idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx, minlength=n)
    expect = m * r["weights"] / r["W"]
    assert np.all(counts >= np.floor(expect - 1e-9)) and np.all(counts <= np.ceil(expect + 1e-9))
    assert counts.sum() == m


def test_sir_estimate_agrees_with_rejection():
    K, bp, c = 8, 40.0, 20.0
    p = OP.plan_point(K, 1.0, bp, c, proposal=1, n_random=0)
    r = oracle.sir(K, 1.0, bp, c, 1, p.alpha_star, p.log_M, 0, 0, 400_000, 10, 0.5)
    s = oracle.sample(K, 1.0, bp, c, 1, p.alpha_star, p.log_M, 7, 0, 2_000_000, 32, cap=0)["stats"]
    assert r["ess"] > 10 * r["W"]                      # far more effective samples than accepts
    assert r["skewness"] == pytest.approx(s.skewness, abs=0.05)
    assert r["kurtosis"] == pytest.approx(s.kurtosis, abs=0.1)
