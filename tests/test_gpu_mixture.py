"""Parity of the gfx950 mixture sampler (learned proposal) with the CPU FP64 oracle.

* per proposal (tkdv_eval_mixture): x^ of the mixture draw (component from the
  same word, in integers), t, log a within the mixture's decision window, and
  the final decision, equal to the oracle's FP64 decision except where
  |log U - log a| < 1e-9;
* end to end (tkdv_sample_mixture): accepted index set, stored rows,
  statistics, accepted-count mode, the policies for a violated rejection
  bound (count, fail, raise M and run again), argument errors.
The mixtures are random (a trained one is not needed for parity): D near the
paper's Sigma, V of rank 2 with entries of size ~1/sqrt(K).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from conftest import check_extremes

pytestmark = pytest.mark.gpu

AMBIG = 1e-9


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


def make_case(T, K, bp, c, scale=1.0, eps=0.2, seed=3, point_id=5, log_M_shift=0.0):
    pt = T.make_point(K, 1.0, bp, c, seed=seed, point_id=point_id)
    sp = T.plan_point(pt, T.SIGMA)
    rng = np.random.default_rng(seed + 100 * K)
    logd = np.log(np.array(sp.sigma2[:K])) + 0.2 * rng.standard_normal(K)
    V = scale * rng.standard_normal((2 * K, 2)) / math.sqrt(K)
    mx = T.make_mixture(K, eps, logd, V)
    mo = oracle.make_mixture(K, eps, logd, V)
    pl, _ = T.plan_mixture(pt, sp, mx, margin=0.02)
    pl.log_M += log_M_shift
    return pt, sp, pl, mx, mo


def oracle_mix(pt, pl, mo, n, i0=0, cap=0):
    return oracle.mix_sample(pt.K, pt.E0, pt.beta_p, pt.c32, pl.alpha_star, pl.log_M, mo, pt.seed,
                             pt.point_id, n, i0=i0, cap=cap, want_log=True)


EVAL_CASES = [  # K, beta', C3/C2, n, i0
    (8, 40.0, 20.0, 4096 + 17, 0),
    (16, 40.0, 60.0, 2048 + 5, 987654321),
    (32, 40.0, 225.0, 1024 + 31, 0),
    (32, 20.0, 450.0, 1024 + 3, (1 << 35) + 11),
]


@pytest.mark.parametrize("K,bp,c,n,i0", EVAL_CASES)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_eval_mixture_against_oracle(T, ctx, K, bp, c, n, i0, prec):
    say(f"eval-mix K={K} beta'={bp} c={c} n={n} i0={i0} prec={prec}")
    pt, sp, pl, mx, mo = make_case(T, K, bp, c)
    P = T.PRECISIONS[prec]
    g = ctx.eval_mixture(pt, pl, mx, i0, n, precision=P)
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = oracle_mix(pt, pl, mo, n, i0=i0)
    draws = [oracle.mix_draw(K, 1.0, bp, c, pl.alpha_star, mo, pt.seed, pt.point_id, i0 + q) for q in range(n)]
    xo = np.stack([d[0] for d in draws])
    comp = np.array([d[1] for d in draws])
    assert (comp < 0).any() and (comp >= 0).any()
    dx = np.linalg.norm(g["xhat"].astype(np.float64) - xo, axis=1)
    say(f"   max |dx^| = {dx.max():.3e}")
    assert dx.max() < 1e-5
    k2 = (np.arange(1, K + 1) ** 2).astype(np.float64)
    to = (xo[:, :K] ** 2 + xo[:, K:] ** 2) @ k2
    assert np.max(np.abs(g["t"] - to) / to) < 2e-5
    tau = T.mixture_window(pt, pl, mx, P)
    err = np.abs(g["log_a"].astype(np.float64) - o["log_a"])
    say(f"   max|dlog a| = {err.max():.3e}, window = {tau:.3e}")
    assert err.max() < tau / 2
    assert np.max(np.abs(g["log_u"] - o["log_u"])) < 1e-6
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    mism = (g["accept"].astype(bool) != o["accept"].astype(bool)) & ~amb
    assert not mism.any(), f"{mism.sum()} decisions differ"


SAMPLE_CASES = [  # K, beta', C3/C2, n, precision, scale
    (8, 40.0, 20.0, 1_000_003, "bf16x3", 1.0),
    (16, 20.0, 60.0, 200_001, "fp32", 0.5),
    (32, 40.0, 75.0, 100_001, "bf16x3", 1.0),
    (32, 20.0, 300.0, 100_003, "fp32", 1.5),
]


@pytest.mark.parametrize("K,bp,c,n,prec,scale", SAMPLE_CASES)
def test_sample_mixture_against_oracle(T, ctx, K, bp, c, n, prec, scale):
    say(f"sample-mix K={K} beta'={bp} c={c} n={n} prec={prec}")
    pt, sp, pl, mx, mo = make_case(T, K, bp, c, scale=scale)
    o = oracle_mix(pt, pl, mo, n, cap=n)
    nacc = int(o["n_accepted"])
    assert nacc > 0
    g = ctx.sample_mixture(pt, pl, mx, n, precision=T.PRECISIONS[prec], capacity=nacc + 8)
    say(f"   accepted gpu={g['n_accepted']} oracle={nacc} fp64 fixups={g['n_fp64_fixups']}")
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    if not amb.any():
        assert g["n_accepted"] == nacc
        assert np.array_equal(g["index"].cpu().numpy().astype(np.uint64), o["index"])
    assert g["n_proposed"] == n and g["n_M_violations"] == int((o["log_a"] > 0).sum())
    xg = g["xhat"].cpu().numpy().astype(np.float64)
    assert np.max(np.linalg.norm(xg - o["xhat"], axis=1)) < 1e-5
    st = oracle.stats_of(o["xhat"], 1.0, 4 * K)
    assert g["n_grid_values"] == st.n_grid
    assert abs(g["S2"] - st.S2) < 1e-5 * st.S2
    assert abs(g["S4"] - st.S4) < 1e-5 * st.S4
    assert abs(g["S3"] - st.S3) < 1e-5 * (st.S2 * math.sqrt(2 * K / math.pi) + 1.0)
    assert g["n_exceed_2sigma"] == st.n_exceed or abs(g["n_exceed_2sigma"] - st.n_exceed) <= 2
    assert np.abs(g["hist_u0"].astype(np.int64) - st.hist.astype(np.int64)).sum() <= 2
    # stats_of indexes the rows; the rows are the accepted proposals in index order
    st.peak_index = int(o["index"][st.peak_index]) if st.n_accepted else st.peak_index
    check_extremes(g, st, 1.0, K, o["xhat"], o["index"])


def test_sample_mixture_accepted_count_mode(T, ctx):
    K, bp, c = 16, 40.0, 60.0
    pt, sp, pl, mx, mo = make_case(T, K, bp, c)
    n_cover = 400_000
    o = oracle_mix(pt, pl, mo, n_cover, cap=n_cover)
    target = int(o["n_accepted"]) // 2
    assert target > 20
    g = ctx.sample_mixture(pt, pl, mx, target, mode=T.COUNT_ACCEPTED, max_proposals=n_cover,
                           precision=T.BF16X3, capacity=target)
    assert g["n_accepted"] == target and g["n_written"] == target
    assert np.array_equal(g["index"].cpu().numpy().astype(np.uint64), o["index"][:target])
    assert g["n_proposed"] == int(o["index"][target - 1]) + 1


def test_sample_mixture_counts_M_violations(T, ctx):
    """An M set too low by 3 nats: every proposal with log a > 0 is counted
    (policy MV_COUNT), or the call fails (MV_FAIL)."""
    K, bp, c = 8, 40.0, 20.0
    pt, sp, pl, mx, mo = make_case(T, K, bp, c, log_M_shift=-3.0)
    n = 300_001
    o = oracle_mix(pt, pl, mo, n)
    nv = int((o["log_a"] > 0).sum())
    assert nv > 0
    try:
        ctx.set_violation_policy(T.MV_COUNT)
        g = ctx.sample_mixture(pt, pl, mx, n, precision=T.FP32)
        assert g["n_M_violations"] == nv and g["M_raises"] == 0
        assert abs(g["max_log_a"] - o["log_a"].max()) < 1e-3
        ctx.set_violation_policy(T.MV_FAIL)
        with pytest.raises(T.TkdvError) as e:
            ctx.sample_mixture(pt, pl, mx, n, precision=T.FP32)
        assert e.value.status == -6
    finally:
        ctx.set_violation_policy(T.MV_RAISE)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_sample_mixture_raises_a_violated_M(T, ctx, prec):
    """The same M, 3 nats too low, under the default policy: log M is raised
    above every log a seen and the point is run again; the result is the
    oracle's run at the raised M (no proposal with f/(M q) > 1)."""
    K, bp, c = 8, 40.0, 20.0
    pt, sp, pl, mx, mo = make_case(T, K, bp, c, log_M_shift=-3.0)
    n = 300_001
    g = ctx.sample_mixture(pt, pl, mx, n, precision=T.PRECISIONS[prec], capacity=n)
    say(f"raised log M {pl.log_M:.6f} -> {g['log_M_used']:.6f} after {g['M_raises']} raise(s)")
    assert g["M_raises"] >= 1 and g["fallback"] == 0 and g["n_M_violations"] == 0
    assert g["log_M_used"] > pl.log_M
    pl2 = type(pl).from_buffer_copy(pl)
    pl2.log_M = g["log_M_used"]
    o = oracle_mix(pt, pl2, mo, n, cap=n)
    assert not (o["log_a"] > 0).any()
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    acc_g = np.zeros(n, dtype=bool)
    acc_g[g["index"].cpu().numpy().astype(np.int64)] = True
    assert not ((acc_g != (o["log_u"] < o["log_a"])) & ~amb).any()
    assert g["n_accepted"] == int(acc_g.sum())


def test_sample_mixture_edges(T, ctx):
    K = 8
    pt, sp, pl, mx, mo = make_case(T, K, 40.0, 20.0)
    g = ctx.sample_mixture(pt, pl, mx, 0)
    assert g["n_proposed"] == 0 and g["n_accepted"] == 0
    g = ctx.sample_mixture(pt, pl, mx, 1, capacity=4)
    o = oracle_mix(pt, pl, mo, 1, cap=1)
    assert g["n_accepted"] == int(o["n_accepted"]) and g["n_proposed"] == 1
    # the Sigma plan is refused, as is K = 64
    with pytest.raises(T.TkdvError):
        ctx.sample_mixture(pt, sp, mx, 1000)
    pt64 = T.make_point(64, 1.0, 40.0, 0.0)
    sp64 = T.plan_point(pt64, T.SIGMA)
    mx64 = T.make_mixture(64, 0.2, np.log(np.array(sp64.sigma2[:64])), np.zeros((128, 2)))
    pl64, _ = T.plan_mixture(pt64, sp64, mx64)
    with pytest.raises(T.TkdvError) as e:
        ctx.sample_mixture(pt64, pl64, mx64, 1000)
    assert e.value.status == -5
    with pytest.raises(T.TkdvError) as e:   # plain BF16 decisions are refused
        ctx.sample_mixture(pt, pl, mx, 1000, precision=T.BF16)
    assert e.value.status == -5
    # with V = 0 and D = Sigma the mixture is the paper's proposal: same law, and
    # the defensive component's draws are the paper's draws index by index
    mx0 = T.make_mixture(K, 0.2, np.log(np.array(sp.sigma2[:K])), np.zeros((2 * K, 2)))
    pl0, _ = T.plan_mixture(pt, sp, mx0)
    assert abs(pl0.log_M - (sp.log_M - sp.log_norm_g)) < 1e-6
