"""The learned proposal's network on the GPU (tkdv_learner_*) against the oracle.

* forward: the network's mixture at a point equals the oracle network's;
* loss and gradients: the per-point loss equals the oracle loss, and the FP64
  kernel gradients dL/d(log d, V) and dL/dweights equal central differences
  of the oracle loss (relative 1e-6);
* training: the trained network's mixture has a smaller rejection constant
  than the untrained one and than the paper's proposal, and the mixture
  sampler then accepts more often while its samples keep the target's law
  (two-sample KS against the paper's sampler).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import learned as OL

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


def random_weights(n, rng, scale=0.3):
    return scale * rng.standard_normal(n)


def test_network_mixture_matches_oracle(T, ctx):
    K, H = 16, 32
    cfg = T.learner_cfg(K, hidden=H, v_amp=0.5, v_scale=0.7)
    L = T.Learner(ctx, cfg)
    rng = np.random.default_rng(1)
    W = random_weights(L.n_weights, rng)
    L.set_weights(W)
    assert np.array_equal(L.get_weights(), W)
    for bp, E0, c in [(30.0, 1.0, 100.0), (45.0, 0.5, 10.0), (20.0, 2.0, 0.0)]:
        pt = T.make_point(K, E0, bp, c)
        sp = T.plan_point(pt, T.SIGMA)
        m = L.mixture(pt, sp)
        o = OL.network(W, H, K, OL.features(bp, E0, c))
        logd, V = OL.mixture_params(o, K, np.array(sp.sigma2[:K]), 0.5, 0.7)
        assert np.allclose(np.array(m.logd[:K]), logd, rtol=0, atol=1e-12)
        Vg = np.array([[m.V[r][q] for q in range(2)] for r in range(2 * K)])
        assert np.allclose(Vg, V, rtol=0, atol=1e-12)
        assert abs(m.eps - 0.2) < 1e-15
    L.close()


def _setup_small(T, ctx, K=8, H=12, seed=2):
    rng = np.random.default_rng(seed)
    cfg = T.learner_cfg(K, hidden=H, eps=0.2, v_amp=0.5, v_scale=0.8, temperature=0.3, nll_weight=0.4)
    L = T.Learner(ctx, cfg)
    W = random_weights(L.n_weights, rng, 0.2)
    L.set_weights(W)
    specs = [(30.0, 1.0, 40.0), (45.0, 1.0, 20.0)]
    pts = [T.make_point(K, E0, bp, c) for bp, E0, c in specs]
    sps = [T.plan_point(p, T.SIGMA) for p in pts]
    L.set_points(pts, sps)
    rows, kinds = [], []
    for i in range(len(pts)):
        X = rng.standard_normal((41, 2 * K))   # more than one chunk of 32 rows
        X /= np.linalg.norm(X, axis=1)[:, None]
        kd = [0] * 20 + [2] * 14 + [1] * 7
        L.add_rows(i, X[:20], kind=0)
        L.add_rows(i, X[20:34], kind=2)
        L.add_rows(i, X[34:], kind=1)
        rows.append(X)
        kinds.append(kd)
    plans = [(sp.alpha_star, np.array(sp.sigma2[:K])) for sp in sps]
    opts = [(E0, bp, c) for bp, E0, c in specs]
    return L, cfg, W, opts, plans, rows, kinds


@pytest.mark.parametrize("K", [8, 16, 32])
def test_loss_and_gradients_against_oracle(T, ctx, K):
    """Loss, dL/d(log d, V) against central differences of the oracle's loss
    for every K of the learner (its matrix-product kernels branch on K), with
    rows of all three kinds over more than one chunk; dL/dweights on a sample
    of coordinates."""
    H = 12
    L, cfg, W, opts, plans, rows, kinds = _setup_small(T, ctx, K, H)
    loss, gmix, gw = L.gradients()
    eps, T_, lam = cfg.eps, cfg.temperature, cfg.nll_weight
    h = 1e-5
    for p, ((E0, bp, c), (a, s2), X, kd) in enumerate(zip(opts, plans, rows, kinds)):
        o = OL.network(W, H, K, OL.features(bp, E0, c))
        logd, V = OL.mixture_params(o, K, s2, cfg.v_amp, cfg.v_scale)
        lo = OL.point_loss(K, E0, bp, c, a, eps, logd, V, X, kd, T_, lam)
        say(f"point {p}: loss gpu {loss[p]:.12f} oracle {lo:.12f}")
        assert abs(loss[p] - lo) < 1e-10 * max(1.0, abs(lo))
        theta = np.concatenate([logd, V.ravel()])
        fd = np.zeros_like(theta)
        for i in range(theta.size):
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            fp = OL.point_loss(K, E0, bp, c, a, eps, tp[:K], tp[K:].reshape(2 * K, 2), X, kd, T_, lam)
            fm = OL.point_loss(K, E0, bp, c, a, eps, tm[:K], tm[K:].reshape(2 * K, 2), X, kd, T_, lam)
            fd[i] = (fp - fm) / (2 * h)
        err = np.abs(gmix[p] - fd)
        say(f"   dL/dtheta max err {err.max():.3e}, max |g| {np.abs(fd).max():.3e}")
        assert np.all(err <= 1e-6 * np.maximum(np.abs(fd), 1e-2))
    # dL/dweights: a sample of coordinates from every block of the layout
    n_out = 5 * K
    blocks = [0, 3 * H, 4 * H, 4 * H + H * H, 5 * H + H * H, 5 * H + H * H + H * n_out]
    rng = np.random.default_rng(3)
    idx = sorted({int(b + rng.integers(0, 5)) for b in blocks} | {int(i) for i in rng.integers(0, L.n_weights, 8)})

    def total(Wv):
        return OL.total_loss(Wv, H, K, opts, plans, rows, kinds, eps, cfg.v_amp, cfg.v_scale, T_, lam)

    for i in idx:
        Wp, Wm = W.copy(), W.copy()
        Wp[i] += h
        Wm[i] -= h
        fd = (total(Wp) - total(Wm)) / (2 * h)
        say(f"   w[{i}]: gpu {gw[i]:.10e} fd {fd:.10e}")
        assert abs(gw[i] - fd) <= 1e-6 * max(abs(fd), 1e-2)
    L.close()


def test_shifted_rows_are_the_oracle_shifts(T, ctx):
    """Rows appended with their xi-shifted copies (rotated on the device) give
    the same loss and gradients as the oracle's shifted rows added directly."""
    K, H = 16, 24
    cfg = T.learner_cfg(K, hidden=H, v_amp=0.5, v_scale=0.7)
    rng = np.random.default_rng(12)
    L0 = T.Learner(ctx, cfg)
    W = random_weights(L0.n_weights, rng)
    L0.close()
    pts = [T.make_point(K, 1.0, 30.0, 100.0), T.make_point(K, 0.5, 45.0, 20.0)]
    sps = [T.plan_point(p, T.SIGMA) for p in pts]
    base = rng.standard_normal((3, 2 * K))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    phis = [0.0, 0.013, 2 * math.pi / 32 * 0.5, 1.7, -2.4]
    losses = []
    for device_shift in (True, False):
        L = T.Learner(ctx, cfg)
        L.set_weights(W)
        L.set_points(pts, sps)
        for i in range(2):
            L.add_rows(i, base[:2], kind=0)
            if device_shift:
                L.add_shifted_rows(i, base, phis, kind=1)
            else:
                rows = np.array([oracle.shift(base[r], ph) for r in range(base.shape[0]) for ph in phis])
                L.add_rows(i, rows, kind=1)
        losses.append(L.gradients())
        L.close()
    (l1, gm1, gw1), (l2, gm2, gw2) = losses
    say(f"shifted rows: loss {l1} vs {l2}")
    assert np.allclose(l1, l2, rtol=1e-12, atol=1e-12)
    assert np.allclose(gm1, gm2, rtol=1e-10, atol=1e-12)
    assert np.allclose(gw1, gw2, rtol=1e-10, atol=1e-12)


def test_training_gains_over_the_paper_proposal(T, ctx):
    """Two K = 16 points; a short fit; the trained network beats both the
    untrained network and the paper's Sigma proposal in M, and the mixture
    sampler's samples follow the same law as the paper's sampler's."""
    from paper_2411_16952_amd import learned
    K = 16
    pts = [T.make_point(K, 1.0, bp, c, seed=5 + i, point_id=i) for i, (bp, c) in enumerate([(30.0, 120.0),
                                                                                           (40.0, 90.0)])]
    cfg = T.learner_cfg(K, hidden=64, v_amp=0.5, v_scale=1.0, lr=3e-3, seed=4)
    res = learned.fit(ctx, pts, cfg, samples_per_point=2048, rounds=6, steps=100, max_proposals=1 << 33, log=say)
    g0 = np.array(res.history[0]["log_gain"])
    g1 = np.array(res.history[res.best_round]["log_gain"])
    say(f"gain M_Sigma/M_mix untrained {np.exp(g0)}, trained {np.exp(g1)}")
    assert np.all(g1 > g0 + math.log(1.5))
    assert np.all(g1 > math.log(2.0))
    # measured acceptance and exactness at the first point
    pt, sp = pts[0], res.sigma_plans[0]
    mix, pl, _ = learned.plan_for(res, pt, margin=0.02)
    n = 1 << 24
    rm = ctx.sample_mixture(pt, pl, mix, n, precision=T.BF16X3, capacity=20000)
    rs = ctx.sample(pt, n, proposal=T.SIGMA, plan=sp, precision=T.BF16X3, capacity=20000)
    say(f"acceptance mixture {rm['acceptance']:.3e} sigma {rs['acceptance']:.3e}, violations {rm['n_M_violations']}")
    assert rm["n_M_violations"] == 0
    assert rm["acceptance"] > 2.0 * rs["acceptance"]
    from scipy import stats
    xm = rm["xhat"].cpu().numpy().astype(np.float64)
    xs = rs["xhat"].cpu().numpy().astype(np.float64)
    assert stats.ks_2samp(xm[:, :K].sum(1), xs[:, :K].sum(1)).pvalue > 0.01
    h3m = np.array([oracle.H3_triad(x / np.linalg.norm(x), 1.0) for x in xm[:3000]])
    h3s = np.array([oracle.H3_triad(x / np.linalg.norm(x), 1.0) for x in xs[:3000]])
    assert stats.ks_2samp(h3m, h3s).pvalue > 0.01
    res.learner.close()


def test_k32_learned_mixture_is_exact(T, ctx):
    """The K = 32 configuration: a network fitted on 16 beta' in [20, 60] at
    C3/C2 = 9000/beta'; at held-out seeds and at C3/C2 = 12000/beta' the
    rejection bound must hold on exact samples of f (the paper's sampler's
    accepted samples: log f - log q_mix - log M_mix <= 0 at every one of them),
    and the mixture sampler's samples must follow the same law (KS on u(0) and
    H3)."""
    from scipy import stats
    from paper_2411_16952_amd import learned
    K = 32
    bps = np.linspace(20, 60, 16)
    pts = [T.make_point(K, 1.0, float(b), 9000.0 / float(b), seed=100 + i, point_id=i) for i, b in enumerate(bps)]
    cfg = T.learner_cfg(K, hidden=256, v_amp=0.5, v_scale=1.0, lr=3e-3, seed=7)
    res = learned.fit(ctx, pts, cfg, samples_per_point=4096, rounds=6, steps=150, max_proposals=1 << 36, log=say)
    # training is deterministic: the same fit gives the same weights bit for bit
    res2 = learned.fit(ctx, pts[:4], cfg, samples_per_point=512, rounds=1, steps=20, max_proposals=1 << 36)
    res3 = learned.fit(ctx, pts[:4], cfg, samples_per_point=512, rounds=1, steps=20, max_proposals=1 << 36)
    assert np.array_equal(res2.learner.get_weights(), res3.learner.get_weights())
    res2.learner.close()
    res3.learner.close()
    for bp, P in [(40.0, 9000.0), (20.0, 12000.0)]:
        pt = T.make_point(K, 1.0, bp, P / bp, seed=4242, point_id=9)
        mix, pl, sp = learned.plan_for(res, pt, margin=0.02)
        gain = math.exp(learned.log_M_sigma_normalised(sp) - pl.log_M)
        rs = ctx.sample(pt, 1 << 31, proposal=T.SIGMA, plan=sp, precision=T.BF16X3, capacity=40000)
        xs = rs["xhat"].cpu().numpy().astype(np.float64)
        xs /= np.linalg.norm(xs, axis=1)[:, None]
        mo = oracle.make_mixture(K, mix.eps, np.array(mix.logd[:K]),
                                 np.array([[mix.V[r][q] for q in range(2)] for r in range(2 * K)]))
        la = np.array([oracle.log_ratio(x, 1.0, bp, P / bp, sp.alpha_star, 0)
                       - oracle.mix_log_q(K, 1.0, bp, P / bp, sp.alpha_star, mo, x)[1] for x in xs]) - pl.log_M
        rm = ctx.sample_mixture(pt, pl, mix, 1 << 28, precision=T.BF16X3, capacity=40000)
        say(f"beta'={bp} P={P}: M gain {gain:.1f}; {len(xs)} exact samples, max log a_mix {la.max():.4f}; "
            f"mixture acc {rm['acceptance']:.3e} (sigma {rs['acceptance']:.3e}), violations {rm['n_M_violations']}")
        assert la.max() <= 0.0, "the rejection bound fails on an exact sample of f"
        assert rm["n_M_violations"] == 0
        xm = rm["xhat"].cpu().numpy().astype(np.float64)
        xm /= np.linalg.norm(xm, axis=1)[:, None]
        p_u0 = stats.ks_2samp(xm[:, :K].sum(1), xs[:, :K].sum(1)).pvalue
        h3m = np.array([oracle.H3_triad(x, 1.0) for x in xm[:len(xs)]])
        h3s = np.array([oracle.H3_triad(x, 1.0) for x in xs])
        p_h3 = stats.ks_2samp(h3m, h3s).pvalue
        say(f"   KS p-values: u(0) {p_u0:.3f}, H3 {p_h3:.3f}")
        assert p_u0 > 0.01 and p_h3 > 0.01
    res.learner.close()
