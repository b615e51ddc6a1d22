"""Oracle of the learned proposal's network and training loss (not in the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy FP64, one
row and one point at a time, written from the definitions:

  features     z = ((beta' - 40)/20, ln E0, (C3/C2) sqrt(E0) beta'/1e4 - 1)
  network      h1 = tanh(W1^T z + b1), h2 = tanh(W2^T h1 + b2), o = W3^T h2 + b3,
               weights in one array, input-major: W1 [3][H], b1 [H], W2 [H][H],
               b2 [H], W3 [H][5K], b3 [5K]
  mixture      log d_k = log s_k^2 + o_{k-1};  V = V0 + v_scale o_{K..5K-1}
               (row-major [2K][2]), V0 = v_amp/sqrt(K) on the cos block of
               column 0 and the sin block of column 1
  loss         L = sum_p [ T log sum_{s in p, kind 0, 1} exp((log f(x_s) - log q_mix(x_s))/T)
                           - lambda mean_{s in p, kind 0, 2} log q_net(x_s) ]
               (kind 0: accepted samples in both terms; kind 1: points where
               f/q_mix is large, soft maximum only; kind 2: accepted samples
               in the likelihood term only)
with log f the unnormalised target of the paper (eq. for f, Sec. III) and
q_net, q_mix the oracle's mixture densities (``core.mix_log_q``).

Pins: the network against a hand-sized case; the loss against its closed
forms (one row: the ratio itself; T -> 0: the maximum); the gradients of the
GPU kernels are compared with central differences of ``total_loss``.
"""
from __future__ import annotations

import math

import numpy as np

from . import core


def features(beta_p: float, E0: float, c32: float) -> np.ndarray:
    return np.array([(beta_p - 40.0) / 20.0, math.log(E0), c32 * math.sqrt(E0) * beta_p / 1e4 - 1.0])


def split_weights(W, H: int, n_out: int):
    W = np.asarray(W, dtype=np.float64)
    o = 0
    W1 = W[o:o + 3 * H].reshape(3, H); o += 3 * H
    b1 = W[o:o + H]; o += H
    W2 = W[o:o + H * H].reshape(H, H); o += H * H
    b2 = W[o:o + H]; o += H
    W3 = W[o:o + H * n_out].reshape(H, n_out); o += H * n_out
    b3 = W[o:o + n_out]; o += n_out
    assert o == W.size, "weight array of the wrong size"
    return W1, b1, W2, b2, W3, b3


def n_weights(H: int, n_out: int) -> int:
    return 5 * H + H * H + H * n_out + n_out


def network(W, H: int, K: int, z) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = split_weights(W, H, 5 * K)
    h1 = np.tanh(z @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    return h2 @ W3 + b3


def mixture_params(o, K: int, sigma2, v_amp: float, v_scale: float):
    """(log d [K], V [2K, 2]) of the network output o [5K]."""
    o = np.asarray(o, dtype=np.float64)
    logd = np.log(np.asarray(sigma2[:K], dtype=np.float64)) + o[:K]
    V0 = np.zeros((2 * K, 2))
    V0[:K, 0] = v_amp / math.sqrt(K)
    V0[K:, 1] = v_amp / math.sqrt(K)
    return logd, V0 + v_scale * o[K:].reshape(2 * K, 2)


def point_loss(K, E0, beta_p, c32, alpha_star, eps, logd, V, rows, kinds, T, lam):
    """Loss of one point for its rows (unit vectors) and kinds (0 accepted
    sample, 1 other point: soft maximum only, 2 accepted sample: likelihood
    only)."""
    m = core.make_mixture(K, eps, logd, V)
    r, nll, n_acc = [], 0.0, 0
    for x, kd in zip(rows, kinds):
        lnet, lmix = core.mix_log_q(K, E0, beta_p, c32, alpha_star, m, x)
        lf = core.log_ratio(x, E0, beta_p, c32, alpha_star, 0)   # log f, unnormalised
        if kd in (0, 1):
            r.append(lf - lmix)
        if kd in (0, 2):
            nll -= lnet
            n_acc += 1
    r = np.array(r) / T
    mx = r.max()
    soft = T * (mx + math.log(np.exp(r - mx).sum()))
    return soft + (lam * nll / n_acc if n_acc else 0.0)


def total_loss(W, H, K, points, plans, rows, kinds, eps, v_amp, v_scale, T, lam):
    """points: (E0, beta', c32) per point; plans: (alpha*, s^2[K]) per point;
    rows/kinds: per point lists."""
    L = 0.0
    for (E0, bp, c), (a, s2), X, kd in zip(points, plans, rows, kinds):
        o = network(W, H, K, features(bp, E0, c))
        logd, V = mixture_params(o, K, s2, v_amp, v_scale)
        L += point_loss(K, E0, bp, c, a, eps, logd, V, X, kd, T, lam)
    return L
