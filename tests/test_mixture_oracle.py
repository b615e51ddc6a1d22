"""Pins of the oracle's learned-proposal functions (not in the paper).

The defensive mixture q_mix = eps g_Sigma + (1 - eps) q_net is built from
angular central Gaussian densities on S^{2K-1}, normalised w.r.t. the uniform
measure mu0.  Each pin below fixes the oracle by something other than its own
formulas:
  * normalisation by quadrature on S^1 (K = 1) and S^3 (K = 2);
  * the dense-matrix definition |L|^{-1/2} (x^T L^{-1} x)^{-K} with explicit
    rotation matrices (numpy slogdet/solve), against the oracle's low-rank
    (Woodbury) evaluation;
  * V = 0, D = Sigma: every component is the paper's g_Sigma (Sec. III.B);
  * invariance of q_net under the S xi-shifts;
  * the draw against the density: E_q[q_net/q_mix] = E_q[g_Sigma/q_mix] = 1
    (importance identities that hold only if the draw has density q_mix);
  * the integer component rule: weight E 2^-32 for g_Sigma, uniform shifts;
  * exactness: the mixture sampler's accepted samples follow the same law
    as the paper's sampler's (two-sample KS), with no M violation.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

S = oracle.MIX_S


def _alpha(K, bp):
    return oracle.alpha_star(K, bp)


def _rot_matrix(K, phi):
    """Matrix of the xi-shift: mode k rotated by the angle k phi (cos block, sin block)."""
    R = np.zeros((2 * K, 2 * K))
    for k in range(1, K + 1):
        c, s = math.cos(k * phi), math.sin(k * phi)
        R[k - 1, k - 1] = c
        R[k - 1, K + k - 1] = s
        R[K + k - 1, K + k - 1] = c
        R[K + k - 1, k - 1] = -s
    return R


def _dense_log_qnet(K, logd, V, x):
    d = np.exp(np.concatenate([logd, logd]))
    L = np.diag(d) + V @ V.T
    _, ld = np.linalg.slogdet(L)
    terms = []
    for j in range(S):
        R = _rot_matrix(K, 2 * math.pi * j / S)
        Lj = R @ L @ R.T
        q = x @ np.linalg.solve(Lj, x)
        terms.append(-0.5 * ld - K * math.log(q))
    terms = np.array(terms)
    m = terms.max()
    return m + math.log(np.exp(terms - m).sum()) - math.log(S)


def _random_mixture(K, rng, scale=0.5, bp=30.0):
    a = _alpha(K, bp)
    s2 = np.array([1.0 / (1.0 + a * bp * k * k / K ** 3) for k in range(1, K + 1)])
    logd = np.log(s2) + 0.2 * rng.standard_normal(K)
    V = scale * rng.standard_normal((2 * K, 2)) / math.sqrt(K)
    return logd, V, a


def _log_g_sigma(K, bp, a, x):
    """The paper's proposal as an ACG: |Sigma|^{-1/2} (x^T Sigma^{-1} x)^{-K}."""
    s2 = np.array([1.0 / (1.0 + a * bp * k * k / K ** 3) for k in range(1, K + 1)])
    d = np.concatenate([s2, s2])
    return -0.5 * np.log(d).sum() - K * math.log((x * x / d).sum())


def test_mixture_normalised_on_circle():
    """K = 1: trapezoid rule in the angle (spectrally exact) integrates q to 1."""
    K, bp = 1, 0.5
    rng = np.random.default_rng(1)
    a = 1.0 / (1.0 - bp)  # root of F at K = 1
    logd = np.array([0.3])
    V = np.array([[0.7, -0.2], [0.1, 0.5]])
    m = oracle.make_mixture(K, 0.2, logd, V)
    th = 2 * math.pi * np.arange(4096) / 4096
    net, mix = [], []
    for t in th:
        ln, lm = oracle.mix_log_q(K, 1.0, bp, 0.0, a, m, [math.cos(t), math.sin(t)])
        net.append(math.exp(ln))
        mix.append(math.exp(lm))
    assert abs(np.mean(net) - 1.0) < 1e-12
    assert abs(np.mean(mix) - 1.0) < 1e-12
    del rng


def test_mixture_normalised_on_three_sphere():
    """K = 2: x^ = (sqrt(1-s) cos a, sqrt(s) cos b | -sqrt(1-s) sin a, -sqrt(s) sin b),
    mu0 = ds da db/(2 pi)^2 on [0,1] x [0,2pi)^2 (Gauss-Legendre in s, trapezoid in angles)."""
    K, bp = 2, 3.0
    rng = np.random.default_rng(2)
    logd, V, a = _random_mixture(K, rng, scale=0.6, bp=bp)
    m = oracle.make_mixture(K, 0.3, logd, V)
    sg, wg = np.polynomial.legendre.leggauss(48)
    sg, wg = 0.5 * (sg + 1.0), 0.5 * wg
    na = 48
    ang = 2 * math.pi * np.arange(na) / na
    tot_net = tot_mix = 0.0
    for s, w in zip(sg, wg):
        r1, r2 = math.sqrt(1 - s), math.sqrt(s)
        for ta in ang:
            for tb in ang:
                x = [r1 * math.cos(ta), r2 * math.cos(tb), -r1 * math.sin(ta), -r2 * math.sin(tb)]
                ln, lm = oracle.mix_log_q(K, 1.0, bp, 0.0, a, m, x)
                tot_net += w * math.exp(ln)
                tot_mix += w * math.exp(lm)
    tot_net /= na * na
    tot_mix /= na * na
    assert abs(tot_net - 1.0) < 1e-8
    assert abs(tot_mix - 1.0) < 1e-8


@pytest.mark.parametrize("K", [3, 8])
def test_mixture_matches_dense_definition(K):
    rng = np.random.default_rng(K)
    logd, V, a = _random_mixture(K, rng, scale=1.2, bp=8.0)
    m = oracle.make_mixture(K, 0.2, logd, V)
    for _ in range(5):
        x = rng.standard_normal(2 * K)
        x /= np.linalg.norm(x)
        ln, _ = oracle.mix_log_q(K, 1.0, 8.0, 0.0, a, m, x)
        assert abs(ln - _dense_log_qnet(K, logd, V, x)) < 1e-11


def test_mixture_with_V0_and_D_sigma_is_g_sigma():
    K, bp = 8, 30.0
    a = _alpha(K, bp)
    s2 = np.array([1.0 / (1.0 + a * bp * k * k / K ** 3) for k in range(1, K + 1)])
    m = oracle.make_mixture(K, 0.25, np.log(s2), np.zeros((2 * K, 2)))
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.standard_normal(2 * K)
        x /= np.linalg.norm(x)
        ln, lm = oracle.mix_log_q(K, 1.0, bp, 0.0, a, m, x)
        ref = _log_g_sigma(K, bp, a, x)
        assert abs(ln - ref) < 1e-12 and abs(lm - ref) < 1e-12


def test_mixture_invariant_under_the_shift_group():
    K = 8
    rng = np.random.default_rng(4)
    logd, V, a = _random_mixture(K, rng, scale=1.0)
    m = oracle.make_mixture(K, 0.2, logd, V)
    x = rng.standard_normal(2 * K)
    x /= np.linalg.norm(x)
    ln0, lm0 = oracle.mix_log_q(K, 1.0, 30.0, 0.0, a, m, x)
    for j in (1, 5, 17):
        y = _rot_matrix(K, 2 * math.pi * j / S) @ x
        ln, lm = oracle.mix_log_q(K, 1.0, 30.0, 0.0, a, m, y)
        assert abs(ln - ln0) < 1e-12 and abs(lm - lm0) < 1e-12
    # a shift off the group changes q_net for a mixture with structure
    y = _rot_matrix(K, 0.37 * 2 * math.pi / S) @ x
    assert abs(oracle.mix_log_q(K, 1.0, 30.0, 0.0, a, m, y)[0] - ln0) > 1e-6


def _draws(K, bp, c, a, m, n, seed=5):
    X, comp = np.zeros((n, 2 * K)), np.zeros(n, dtype=int)
    for i in range(n):
        X[i], comp[i], _ = oracle.mix_draw(K, 1.0, bp, c, a, m, seed, 0, i)
    return X, comp


def test_mixture_draw_has_density_q_mix():
    """E_q[q_net/q_mix] = E_mu0[q_net] = 1 and E_q[g_Sigma/q_mix] = 1: bounded ratios
    (<= 1/(1 - eps) and <= 1/eps), so the Monte Carlo error is controlled."""
    K, bp, n = 8, 30.0, 20000
    rng = np.random.default_rng(6)
    logd, V, a = _random_mixture(K, rng, scale=4.0, bp=bp)
    m = oracle.make_mixture(K, 0.3, logd, V)
    X, _ = _draws(K, bp, 0.0, a, m, n)
    r_net, r_g = np.zeros(n), np.zeros(n)
    for i in range(n):
        ln, lm = oracle.mix_log_q(K, 1.0, bp, 0.0, a, m, X[i])
        r_net[i] = math.exp(ln - lm)
        r_g[i] = math.exp(_log_g_sigma(K, bp, a, X[i]) - lm)
    for r in (r_net, r_g):
        se = r.std() / math.sqrt(n)
        assert abs(r.mean() - 1.0) < 5 * se + 1e-3, (r.mean(), se)
    # and it fails for draws of another mixture (the identity is informative)
    m2 = oracle.make_mixture(K, 0.3, logd, 0.5 * V)
    X2, _ = _draws(K, bp, 0.0, a, m2, 5000)
    r2 = np.array([math.exp(np.subtract(*oracle.mix_log_q(K, 1.0, bp, 0.0, a, m, x))) for x in X2])
    assert abs(r2.mean() - 1.0) > 10 * r2.std() / math.sqrt(5000)


def test_mixture_component_weights():
    K, n = 8, 40000
    rng = np.random.default_rng(7)
    logd, V, a = _random_mixture(K, rng)
    m = oracle.make_mixture(K, 0.2, logd, V)
    eps = oracle.mix_eps(m)
    assert eps == oracle.mix_threshold(m) / 2.0 ** 32 and abs(eps - 0.2) < 2.0 ** -27 * S
    _, comp = _draws(K, 30.0, 0.0, a, m, n)
    nd = int((comp < 0).sum())
    assert abs(nd - eps * n) < 5 * math.sqrt(n * eps * (1 - eps))
    counts = np.bincount(comp[comp >= 0], minlength=S)
    assert counts.size == S
    assert stats.chisquare(counts).pvalue > 1e-3


def test_mixture_sampler_is_exact():
    """Accepted samples of the mixture sampler and of the paper's sampler: same law."""
    K, bp, c = 8, 40.0, 20.0
    pl = oracle.plan_point(K, 1.0, bp, c, 1, seed=0)
    rng = np.random.default_rng(8)
    logd, V, a = _random_mixture(K, rng, scale=0.8, bp=bp)
    m = oracle.make_mixture(K, 0.2, logd, V)
    # M_mix: sup of log f - log q_mix over the plain sampler's best points and random
    # starts, by Nelder-Mead on the sphere; then a margin
    from scipy import optimize

    def neg(y):
        x = y / np.linalg.norm(y)
        lf = oracle.log_ratio(x, 1.0, bp, c, a, 0)
        return -(lf - oracle.mix_log_q(K, 1.0, bp, c, a, m, x)[1])

    starts = [np.r_[np.ones(K), np.zeros(K)] / math.sqrt(K)] + [rng.standard_normal(2 * K) for _ in range(6)]
    best = max(-optimize.minimize(neg, s0, method="Nelder-Mead",
                                  options=dict(maxiter=40000, xatol=1e-10, fatol=1e-13)).fun for s0 in starts)
    log_M = best + math.log(1.05)
    n = 600000
    res_m = oracle.mix_sample(K, 1.0, bp, c, a, log_M, m, 11, 0, n, cap=n, want_log=True)
    assert res_m["log_a"].max() < 0.0  # no M violation
    res_s = oracle.sample(K, 1.0, bp, c, 1, pl.alpha_star, pl.log_M, 12, 0, n, 4 * K, cap=n)
    xm, xs = res_m["xhat"], res_s["xhat"]
    assert len(xm) > 300 and len(xs) > 300
    u0m, u0s = xm[:, :K].sum(1), xs[:, :K].sum(1)
    h3m = np.array([oracle.H3_triad(x, 1.0) for x in xm])
    h3s = np.array([oracle.H3_triad(x, 1.0) for x in xs])
    assert stats.ks_2samp(u0m, u0s).pvalue > 0.01
    assert stats.ks_2samp(h3m, h3s).pvalue > 0.01
