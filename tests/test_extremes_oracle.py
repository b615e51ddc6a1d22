"""Pins of the oracle's extreme-wave search (oracle.extremes), no GPU.

* The zero-mean Dirichlet kernel (equal cos coefficients, Sec. IV.A) attains
  the largest displacement any unit x^ can have, u(0) = sqrt(2 K E0/pi)
  (Cauchy-Schwarz), at xi = 0, i.e. grid index N/2.
* A single cos mode k has maximum sqrt(2 E0/pi) at the first grid point with
  k xi_j = 0 mod 2 pi: j = N/2 for k = 1, j = 0 for k = 2 (xi_0 = -pi).
* Shifting every mode by one grid step (mode k rotated by k 2 pi/N) rolls the
  grid values by one index: the maximum is unchanged and its index moves by
  one (mod N).
* The maximum of -x^ is minus the minimum of x^.
* The first sin mode peaks at xi = +pi/2 (pins the sign of the sin block).
* Ranking: descending maxima, ties by lower row; the exceedance count.
"""
import math

import numpy as np
import pytest

import oracle


def dirichlet(K):
    x = np.zeros(2 * K)
    x[:K] = 1.0 / math.sqrt(K)
    return x


def shift_one_step(x, N):
    K = x.size // 2
    k = np.arange(1, K + 1)
    phi = 2 * math.pi / N
    a, b = x[:K], x[K:]
    # u(xi) -> u(xi - phi): a_k cos k(xi - phi) + b_k sin k(xi - phi)
    c, s = np.cos(k * phi), np.sin(k * phi)
    return np.concatenate([a * c - b * s, b * c + a * s])


@pytest.mark.parametrize("K,E0", [(8, 1.0), (16, 2.0), (32, 0.5), (64, 1.0), (128, 1.5)])
def test_dirichlet_kernel_is_the_largest_wave(K, E0):
    N = 4 * K
    rng = np.random.default_rng(K)
    rows = rng.standard_normal((200, 2 * K))
    rows /= np.linalg.norm(rows, axis=1, keepdims=True)
    rows[57] = dirichlet(K)
    r = oracle.extremes(rows, E0, N, 5, 4 * math.sqrt(E0 / math.pi))
    assert r["rows"][0] == 57
    assert r["umax"][57] == pytest.approx(math.sqrt(2 * K * E0 / math.pi), rel=1e-13)
    assert r["jmax"][57] == N // 2
    assert np.all(r["umax"] <= math.sqrt(2 * K * E0 / math.pi) * (1 + 1e-13))


@pytest.mark.parametrize("K", [8, 32, 128])
def test_single_modes(K):
    N = 4 * K
    amp = math.sqrt(2 / math.pi)
    x1 = np.zeros(2 * K); x1[0] = 1.0
    x2 = np.zeros(2 * K); x2[1] = 1.0
    r = oracle.extremes(np.array([x1, x2]), 1.0, N, 2, 0.0)
    assert r["umax"] == pytest.approx([amp, amp], rel=1e-14)
    assert list(r["jmax"]) == [N // 2, 0]
    assert list(r["rows"]) == [0, 1]          # equal maxima: lower row first
    assert r["n_exceed"] == 2


def test_one_grid_step_shift_rolls_the_argmax():
    K, N = 16, 64
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = rng.standard_normal(2 * K)
        x /= np.linalg.norm(x)
        a = oracle.extremes(x[None], 1.0, N, 1, 0.0)
        b = oracle.extremes(shift_one_step(x, N)[None], 1.0, N, 1, 0.0)
        assert b["umax"][0] == pytest.approx(a["umax"][0], abs=1e-13)
        assert b["jmax"][0] == (a["jmax"][0] + 1) % N


def test_negation_maps_max_to_minus_min():
    K, N = 8, 32
    rng = np.random.default_rng(4)
    x = rng.standard_normal((10, 2 * K))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    r = oracle.extremes(-x, 1.0, N, 10, 0.0)
    for i in range(10):
        assert r["umax"][i] == pytest.approx(-oracle.grid(x[i], 1.0, N).min(), abs=1e-14)


def test_ranking_and_exceedance():
    K, N = 8, 32
    rng = np.random.default_rng(5)
    x = rng.standard_normal((300, 2 * K))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x[10] = x[200]                             # a tie: row 10 before row 200
    thr = 1.5
    r = oracle.extremes(x, 1.0, N, 300, thr)
    um = r["umax"]
    order = list(r["rows"])
    assert all(um[order[i]] >= um[order[i + 1]] for i in range(len(order) - 1))
    assert order.index(10) == order.index(200) - 1
    assert r["n_exceed"] == sum(1 for v in um if v > thr)


def test_sin_mode_position_pins_the_sin_block_sign():
    """u = amp sin(xi) for the first sin mode peaks at xi = +pi/2 (j = 3N/4);
    a sign slip in the sin block would put it at xi = -pi/2 (j = N/4)."""
    K, N = 16, 64
    x = np.zeros(2 * K); x[K] = 1.0
    r = oracle.extremes(x[None], 1.0, N, 1, 0.0)
    assert r["jmax"][0] == 3 * N // 4
    assert r["umax"][0] == pytest.approx(math.sqrt(2 / math.pi), rel=1e-14)
    assert oracle.extremes(-x[None], 1.0, N, 1, 0.0)["jmax"][0] == N // 4
