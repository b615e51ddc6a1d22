"""Pins of the oracle of the learned proposal's network and loss (CPU).

* the flat weight layout, by a one-hidden-unit network whose output is a
  scalar chain of tanh evaluated by hand;
* a zero output layer gives the base mixture D = Sigma, V = V0;
* the loss of a point with one row is log f - log q_mix at that row, and
  as T -> 0 the soft maximum tends to the largest ratio.
"""
import math

import numpy as np

import oracle
from oracle import learned as OL


def test_network_layout_one_hidden_unit():
    K, H = 2, 1
    n_out = 5 * K
    W = np.zeros(OL.n_weights(H, n_out))
    # W1[c][0] at index c, b1 at 3, W2[0][0] at 4, b2 at 5, W3[0][o] at 6 + o, b3 at 6 + n_out + o
    W[0], W[1], W[2], W[3] = 0.3, -0.7, 0.2, 0.1
    W[4], W[5] = 1.3, -0.2
    W[6:6 + n_out] = np.linspace(-1, 1, n_out)
    W[6 + n_out:] = 0.05
    z = OL.features(30.0, 2.0, 50.0)
    assert np.allclose(z, [-0.5, math.log(2.0), 50.0 * math.sqrt(2.0) * 30.0 / 1e4 - 1.0])
    h1 = math.tanh(0.3 * z[0] - 0.7 * z[1] + 0.2 * z[2] + 0.1)
    h2 = math.tanh(1.3 * h1 - 0.2)
    want = np.linspace(-1, 1, n_out) * h2 + 0.05
    assert np.allclose(OL.network(W, H, K, z), want, rtol=0, atol=1e-15)


def test_zero_output_layer_gives_base_mixture():
    K, H = 8, 4
    rng = np.random.default_rng(0)
    W = rng.standard_normal(OL.n_weights(H, 5 * K))
    W[5 * H + H * H:] = 0.0  # W3 and b3
    o = OL.network(W, H, K, OL.features(40.0, 1.0, 20.0))
    s2 = np.linspace(0.5, 0.1, K)
    logd, V = OL.mixture_params(o, K, s2, 0.5, 1.0)
    assert np.allclose(logd, np.log(s2))
    assert np.allclose(V[:K, 0], 0.5 / math.sqrt(K)) and np.allclose(V[K:, 1], 0.5 / math.sqrt(K))
    assert np.all(V[K:, 0] == 0) and np.all(V[:K, 1] == 0)


def test_loss_closed_forms():
    K, bp, c = 8, 40.0, 20.0
    a = oracle.alpha_star(K, bp)
    s2 = oracle.sigma2(K, bp, a)
    rng = np.random.default_rng(1)
    logd = np.log(s2) + 0.1 * rng.standard_normal(K)
    V = 0.3 * rng.standard_normal((2 * K, 2))
    X = rng.standard_normal((6, 2 * K))
    X /= np.linalg.norm(X, axis=1)[:, None]
    m = oracle.make_mixture(K, 0.2, logd, V)
    r = []
    for x in X:
        lf = oracle.log_ratio(x, 1.0, bp, c, a, 0)
        r.append(lf - oracle.mix_log_q(K, 1.0, bp, c, a, m, x)[1])
    one = OL.point_loss(K, 1.0, bp, c, a, 0.2, logd, V, X[:1], [1], 0.05, 0.0)
    assert abs(one - r[0]) < 1e-12
    cold = OL.point_loss(K, 1.0, bp, c, a, 0.2, logd, V, X, [1] * 6, 1e-4, 0.0)
    assert abs(cold - max(r)) < 1e-3
    # the likelihood term: mean of -log q_net over kind-0 rows
    lam = 0.7
    with_nll = OL.point_loss(K, 1.0, bp, c, a, 0.2, logd, V, X[:1], [0], 0.05, lam)
    assert abs(with_nll - r[0] + lam * oracle.mix_log_q(K, 1.0, bp, c, a, m, X[0])[0]) < 1e-12
    # kind 2 (likelihood only): absent from the soft maximum, present in the mean
    lq = [oracle.mix_log_q(K, 1.0, bp, c, a, m, x)[0] for x in X]
    mixed = OL.point_loss(K, 1.0, bp, c, a, 0.2, logd, V, X[:3], [1, 2, 2], 0.05, lam)
    assert abs(mixed - (r[0] - lam * (lq[1] + lq[2]) / 2)) < 1e-12
    both = OL.point_loss(K, 1.0, bp, c, a, 0.2, logd, V, X[:2], [0, 2], 0.05, lam)
    assert abs(both - (r[0] - lam * (lq[0] + lq[1]) / 2)) < 1e-12
