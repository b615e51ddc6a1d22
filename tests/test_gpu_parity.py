"""Parity of the gfx950 sampler with the CPU FP64 oracle, through the C ABI.

* per proposal (tkdv_eval_proposals): x^ after Box-Muller and projection, t,
  the grid sum of cubes S3, log a (within the decision window, which bounds
  the fast path's error) and the final accept decision, which must equal the
  oracle's FP64 decision except where |log U - log a| < 1e-9;
* end to end (tkdv_sample / tkdv_sample_batch): the accepted index set, the
  stored rows of x^, and the statistics, in proposal-count and accepted-count
  modes, with capacity truncation, ragged tails and several K in one batch.
Sizes span many 32-proposal tiles and a ragged tail while the oracle finishes
in seconds.
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


def oracle_run(pt, plan, proposal, n, i0=0, cap=0, want_log=True):
    K = pt.K
    return oracle.sample(K, pt.E0, pt.beta_p, pt.c32, proposal, plan.alpha_star, plan.log_M,
                         pt.seed, pt.point_id, n, 4 * K, i0=i0, cap=cap, want_log=want_log)


def oracle_S3(xhat):
    """sum_j u~_j^3 on the N = 4K grid from the oracle's FP64 H3 (definition of H3):
    H3 = (pi/(3N)) (2 E0/pi)^{3/2} S3 at E0 = 1/scale-free form with amp = 1."""
    K = xhat.shape[1] // 2
    out = np.empty(xhat.shape[0])
    for r in range(xhat.shape[0]):
        u = oracle.grid(xhat[r], math.pi / 2, 4 * K)  # E0 = pi/2 gives amp = 1: u = u~
        out[r] = np.sum(u ** 3)
    return out


EVAL_CASES = [  # K, beta', C3/C2, proposal, n, i0
    (8, 40.0, 20.0, 1, 4096 + 17, 0),
    (16, 40.0, 60.0, 1, 2048 + 5, 123456789),
    (32, 40.0, 150.0, 1, 1024 + 31, 0),
    (32, 20.0, 300.0, 0, 1024 + 3, (1 << 33) + 7),
    (64, 40.0, 300.0, 1, 512 + 9, 0),
    (64, 20.0, 150.0, 0, 256 + 7, 1 << 20),   # the quarter-period kernel with the uniform proposal
]


@pytest.mark.parametrize("K,bp,c,prop,n,i0", EVAL_CASES)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_eval_proposals_against_oracle(T, ctx, K, bp, c, prop, n, i0, prec):
    say(f"eval K={K} beta'={bp} c={c} prop={prop} n={n} i0={i0} prec={prec}")
    pt = T.make_point(K, 1.0, bp, c, seed=11, point_id=3)
    plan = T.plan_point(pt, prop)
    P = T.PRECISIONS[prec]
    g = ctx.eval_proposals(pt, i0, n, proposal=prop, plan=plan, precision=P)
    g = {k: v.cpu().numpy() for k, v in g.items()}
    o = oracle_run(pt, plan, prop, n, i0=i0)
    xo = np.stack([oracle.proposal(K, 1.0, bp, c, prop, plan.alpha_star, plan.log_M, 11, 3, i0 + q)[0]
                   for q in range(n)])
    # x^: FP32 Box-Muller and projection against FP64
    dx = np.linalg.norm(g["xhat"].astype(np.float64) - xo, axis=1)
    assert dx.max() < 2e-6, f"max |dx^|_2 = {dx.max():.3e}"
    # t = sum k^2 s_k
    k2 = (np.arange(1, K + 1) ** 2).astype(np.float64)
    to = (xo[:, :K] ** 2 + xo[:, K:] ** 2) @ k2
    assert np.max(np.abs(g["t"] - to) / to) < 1e-5
    # S3 = sum_j u~_j^3: error bound of the synthesis arithmetic
    s3o = oracle_S3(xo)
    # |dS3| <= 3 (N/2) max_j|du~_j| + FP32 accumulation, max|du~| <= sqrt(K)(eps_prod + |dx^|)
    N = 4 * K
    # per-product error of the arithmetic (x = hi + lo + d, |d| <= 2^-18 |x| for
    # BF16x3) plus FP32 accumulation of 2K products
    eps = {"fp32": 0.0, "bf16x3": 3.02 * 2.0**-18}[prec] + 2 * K * 2.0**-23
    bound = 3 * (N / 2) * np.sqrt(K) * (eps + dx.max()) + N * 2.0**-23 * np.sqrt(K) * N / 2
    ds3 = np.abs(g["s3"] - s3o)
    say(f"   max|dS3| = {ds3.max():.3e}, bound = {bound:.3e}")
    assert ds3.max() < bound
    # log a within the decision window (a bound on the fast path's error)
    tau = T.decision_window(pt, prop, P)
    err = np.abs(g["log_a"].astype(np.float64) - o["log_a"])
    say(f"   max|dlog a| = {err.max():.3e}, window = {tau:.3e}")
    assert err.max() < tau / 2
    assert np.max(np.abs(g["log_u"] - o["log_u"])) < 1e-6
    # decisions: identical to the FP64 oracle except within 1e-9 of the threshold
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    mism = (g["accept"].astype(bool) != o["accept"].astype(bool)) & ~amb
    assert not mism.any(), f"{mism.sum()} decisions differ"


SAMPLE_CASES = [  # K, beta', C3/C2, proposal, n, precision
    (8, 40.0, 20.0, 1, 1_000_000, "bf16x3"),   # the CPU-sized configuration, Sigma proposal
    (8, 40.0, 20.0, 0, 1_000_000, "bf16x3"),   # ... and the uniform proposal
    (16, 20.0, 60.0, 1, 200_003, "fp32"),
    (32, 40.0, 75.0, 1, 100_001, "bf16x3"),
    (64, 40.0, 300.0, 1, 20_011, "fp32"),
]


@pytest.mark.parametrize("K,bp,c,prop,n,prec", SAMPLE_CASES)
def test_sample_matches_oracle(T, ctx, K, bp, c, prop, n, prec):
    say(f"sample K={K} beta'={bp} c={c} prop={prop} n={n} prec={prec}")
    pt = T.make_point(K, 1.0, bp, c, seed=0, point_id=0)
    plan = T.plan_point(pt, prop)
    cap = 200_000
    r = ctx.sample(pt, n, proposal=prop, plan=plan, precision=T.PRECISIONS[prec], capacity=cap)
    o = oracle_run(pt, plan, prop, n, cap=cap)
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    acc_o = o["accept"].astype(bool)
    idx_g = r["index"].cpu().numpy().astype(np.int64)
    acc_g = np.zeros(n, dtype=bool)
    acc_g[idx_g] = True
    assert not ((acc_g != acc_o) & ~amb).any()
    assert r["n_proposed"] == n
    assert r["n_accepted"] == acc_g.sum() == len(idx_g)
    assert np.all(np.diff(idx_g) > 0), "accepted samples must be in increasing proposal index"
    # stored rows equal the oracle's x^ of the same proposals
    same = np.isin(idx_g, o["index"])
    xg = r["xhat"].cpu().numpy().astype(np.float64)[same]
    xo = o["xhat"][np.isin(o["index"], idx_g)]
    assert np.max(np.linalg.norm(xg - xo, axis=1)) < 2e-6
    # statistics: FP64 moments of an FP32 synthesis, integer counts exact up to
    # values within rounding of a bin edge / the 2-sigma level
    so = o["stats"]
    if so.n_accepted > 0:
        for name in ("S2", "S4"):
            assert r[name] == pytest.approx(getattr(so, name), rel=2e-5)
        for name in ("S1", "S3"):
            assert abs(r[name] - getattr(so, name)) < 2e-5 * so.S2 ** (1 if name == "S1" else 1.5) + 1e-9
        assert r["n_grid_values"] == so.n_grid
        assert abs(int(r["n_exceed_2sigma"]) - int(so.n_exceed)) <= 2 + so.n_exceed // 100000
        assert np.abs(r["hist_u0"].astype(np.int64) - so.hist.astype(np.int64)).sum() <= 2
    check_extremes(r, so, 1.0, K, o["xhat"], o["index"])
    assert r["n_M_violations"] == so.n_violations == 0


def test_accepted_count_mode(T, ctx):
    say("accepted-count mode K=16")
    pt = T.make_point(16, 1.0, 40.0, 30.0, seed=5, point_id=2)
    plan = T.plan_point(pt, T.SIGMA)
    target = 1500
    r = ctx.sample(pt, target, proposal=T.SIGMA, plan=plan, mode=T.COUNT_ACCEPTED,
                   max_proposals=10_000_000, capacity=target, precision=T.BF16X3)
    o = oracle.sample_until(16, 1.0, 40.0, 30.0, 1, plan.alpha_star, plan.log_M, 5, 2, target, 10_000_000, 64)
    assert r["n_accepted"] == target
    assert np.array_equal(r["index"].cpu().numpy().astype(np.uint64), o["index"])
    assert r["n_proposed"] == o["stats"].n_proposed
    assert r["S2"] == pytest.approx(o["stats"].S2, rel=2e-5)
    assert np.abs(r["hist_u0"].astype(np.int64) - o["stats"].hist.astype(np.int64)).sum() <= 2
    check_extremes(r, o["stats"], 1.0, 16, o["xhat"], o["index"])


def test_capacity_truncates_rows_not_statistics(T, ctx):
    say("capacity truncation")
    pt = T.make_point(8, 1.0, 40.0, 20.0, seed=3, point_id=1)
    plan = T.plan_point(pt, T.SIGMA)
    full = ctx.sample(pt, 300_000, plan=plan, capacity=100_000)
    part = ctx.sample(pt, 300_000, plan=plan, capacity=100)
    assert part["n_written"] == 100 and full["n_written"] == full["n_accepted"] > 100
    assert np.array_equal(part["index"].cpu().numpy(), full["index"][:100].cpu().numpy())
    assert np.array_equal(part["xhat"].cpu().numpy(), full["xhat"][:100].cpu().numpy())
    assert part["S3"] == full["S3"] and part["n_accepted"] == full["n_accepted"]


@pytest.mark.parametrize("n", [1, 31, 32, 33, 65536 + 1])
def test_ragged_sizes_and_determinism(T, ctx, n):
    say(f"ragged n={n}")
    pt = T.make_point(8, 1.0, 0.0, 0.0, seed=9, point_id=4)  # beta' = 0: every proposal accepted
    plan = T.plan_point(pt, T.SIGMA)
    r1 = ctx.sample(pt, n, plan=plan, capacity=n)
    r2 = ctx.sample(pt, n, plan=plan, capacity=n)
    assert r1["n_accepted"] == n
    assert np.array_equal(r1["index"].cpu().numpy(), np.arange(n))
    assert np.array_equal(r1["xhat"].cpu().numpy(), r2["xhat"].cpu().numpy())
    assert r1["S4"] == r2["S4"]
    assert r1["S2"] / r1["n_grid_values"] == pytest.approx(1 / math.pi, rel=1e-6)


def test_batch_equals_single_point_runs(T, ctx):
    say("batch of mixed K")
    specs = [(8, 40.0, 20.0, 100_000), (16, 40.0, 30.0, 70_001), (32, 40.0, 75.0, 40_000), (8, 20.0, 0.0, 5_000)]
    pts = [T.make_point(K, 1.0, bp, c, seed=21, point_id=p) for p, (K, bp, c, _) in enumerate(specs)]
    plans = [T.plan_point(p, T.SIGMA) for p in pts]
    ns = [s[3] for s in specs]
    caps = [50_000] * len(specs)
    out, _, _ = ctx.sample_batch(pts, ns, plans=plans, capacity=caps)
    for p in range(len(specs)):
        single = ctx.sample(pts[p], ns[p], plan=plans[p], capacity=caps[p])
        assert out[p]["n_accepted"] == single["n_accepted"]
        assert np.array_equal(out[p]["index"].cpu().numpy(), single["index"].cpu().numpy())
        assert np.array_equal(out[p]["xhat"].cpu().numpy(), single["xhat"].cpu().numpy())
        assert out[p]["S3"] == single["S3"]
        assert np.array_equal(out[p]["hist_u0"], single["hist_u0"])


@pytest.mark.parametrize("K,bp,c,n", [(16, 40.0, 60.0, 200_003), (64, 40.0, 150.0, 100_003),
                                     (128, 40.0, 750.0, 100_003)])
def test_sample_raises_a_violated_M(T, ctx, K, bp, c, n):
    """A Sigma plan whose log M is set half a nat below the largest log a of the
    proposals: under the default policy the sampler raises log M above every
    log a seen and runs the point again, which then equals the oracle at the
    raised M; the batch call does the same for the violating point only (the
    half-period kernel at K = 16, the quarter-period kernel at K = 64, 128)."""
    pt = T.make_point(K, 1.0, bp, c, seed=5, point_id=9)
    plan = T.plan_point(pt, T.SIGMA)
    pilot = ctx.sample(pt, n, plan=plan, precision=T.BF16X3)
    assert pilot["n_M_violations"] == 0 and pilot["M_raises"] == 0
    low = type(plan).from_buffer_copy(plan)
    low.log_M += pilot["max_log_a"] - 0.5
    r = ctx.sample(pt, n, plan=low, precision=T.BF16X3, capacity=n)
    say(f"raised log M {low.log_M:.5f} -> {r['log_M_used']:.5f} after {r['M_raises']} raise(s)")
    assert r["M_raises"] >= 1 and r["n_M_violations"] == 0 and r["log_M_used"] > low.log_M
    hi = type(plan).from_buffer_copy(plan)
    hi.log_M = r["log_M_used"]
    o = oracle_run(pt, hi, T.SIGMA, n, cap=n)
    assert not (o["log_a"] > 0).any()
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    acc_g = np.zeros(n, dtype=bool)
    acc_g[r["index"].cpu().numpy().astype(np.int64)] = True
    assert not ((acc_g != o["accept"].astype(bool)) & ~amb).any()
    pt2 = T.make_point(K, 1.0, bp, 0.5 * c, seed=5, point_id=10)
    plan2 = T.plan_point(pt2, T.SIGMA)
    out, _, _ = ctx.sample_batch([pt, pt2], [n, n], plans=[low, plan2], precision=T.BF16X3, capacity=[n, n])
    assert out[0]["M_raises"] == r["M_raises"] and out[0]["log_M_used"] == r["log_M_used"]
    assert out[0]["n_accepted"] == r["n_accepted"] and out[1]["M_raises"] == 0
    assert np.array_equal(out[0]["index"].cpu().numpy(), r["index"].cpu().numpy())
    # the other policies at the low M: counted (every proposal whose FP64 log a
    # is above 0 by more than the fast path's error, at most those above 0), or
    # the call fails
    o_low = oracle_run(pt, low, T.SIGMA, n, cap=0)
    try:
        ctx.set_violation_policy(T.MV_COUNT)
        g = ctx.sample(pt, n, plan=low, precision=T.BF16X3)
        say(f"counted {g['n_M_violations']} violations; oracle: {(o_low['log_a'] > 0).sum()} above 0")
        assert (o_low["log_a"] > 1e-2).sum() <= g["n_M_violations"] <= (o_low["log_a"] > 0).sum()
        assert g["M_raises"] == 0 and g["log_M_used"] == low.log_M
        ctx.set_violation_policy(T.MV_FAIL)
        with pytest.raises(T.TkdvError) as e:
            ctx.sample(pt, n, plan=low, precision=T.BF16X3)
        assert e.value.status == -6
    finally:
        ctx.set_violation_policy(T.MV_RAISE)


@pytest.mark.parametrize("K,bp", [(8, 20.0), (16, 20.0), (32, 60.0), (64, 40.0), (128, 40.0)])
def test_exact_M_is_kept_at_linear_points(T, ctx, K, bp):
    """C3/C2 = 0: log M is the closed form, the exact supremum, so f/(M g) <= 1
    holds everywhere and no proposal may count as a violation.  Near the
    maximiser the fast path's log a can round above 0 by a few ulps; those
    proposals are settled in FP64, M is kept (no raise), and the accepted set
    is the oracle's at that M (acceptance 0.8-0.99 here, so nearly every
    proposal's decision is compared)."""
    n = 100_003
    pt = T.make_point(K, 1.0, bp, 0.0, seed=21, point_id=4)
    plan = T.plan_point(pt, T.SIGMA)
    assert plan.M_source == 0
    r = ctx.sample(pt, n, plan=plan, precision=T.BF16X3, capacity=n)
    say(f"K={K} beta'={bp}: accepted {r['n_accepted']} of {n}, max fast-path log a {r['max_log_a']:.2e}, "
        f"raises {r['M_raises']}, FP64 re-decisions {r['n_fp64_fixups']}")
    assert r["M_raises"] == 0 and r["n_M_violations"] == 0 and r["log_M_used"] == plan.log_M
    o = oracle_run(pt, plan, T.SIGMA, n, cap=n)
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    acc_g = np.zeros(n, dtype=bool)
    acc_g[r["index"].cpu().numpy().astype(np.int64)] = True
    assert not ((acc_g != o["accept"].astype(bool)) & ~amb).any()


def test_invalid_arguments_are_rejected(T, ctx):
    with pytest.raises(T.TkdvError) as e:
        ctx.sample(T.make_point(12, 1.0, 10.0, 1.0), 100)
    assert e.value.status == -5
    with pytest.raises(T.TkdvError) as e:
        ctx.sample(T.make_point(8, 1.0, 10.0, 1.0), 100, mode=T.COUNT_ACCEPTED, max_proposals=0)
    assert e.value.status == -1
    # plain BF16 products miss the 1e-3 tolerance on H3: no decision is taken with them
    pt = T.make_point(32, 1.0, 40.0, 75.0)
    with pytest.raises(T.TkdvError) as e:
        ctx.sample(pt, 1000, precision=T.BF16)
    assert e.value.status == -5
    with pytest.raises(T.TkdvError) as e:
        ctx.eval_proposals(pt, 0, 64, precision=T.BF16)
    assert e.value.status == -5
    with pytest.raises(T.TkdvError) as e:
        ctx.sample_batch([pt], [1000], precision=T.BF16)
    assert e.value.status == -5
