"""K = 128 (N = 512) on the GPU against the CPU FP64 oracle, through the C ABI.

The paper's largest mode count (its parallel speed-up study, Sec. V.C, and
alpha* of Fig. 1) runs in its own kernels: 16 proposals per wavefront, four
lanes each, and the grid sum of cubes behind H3 formed from a quarter of the
grid offset by half a step (cos/sin blocks and even/odd modes synthesised
separately on 16x16x32 BF16 or 16x16x4 FP32 matrix instructions).

* per proposal (tkdv_eval_proposals): x^, t, S3 = the grid sum of cubes (the
  offset grid's sum equals the standard grid's: both are (3N/pi) H3 exactly),
  log a within half the decision window, log U, and the decision, equal to the
  oracle's FP64 decision except within 1e-9 of the threshold; over 2^16
  proposals the worst-case H3 error against the cube-sum scale is below 1e-6
  (FP32) and 1e-5 (BF16x3), and H = H2 - (C3/C2) H3 agrees to 1e-6 relative;
* end to end (tkdv_sample, tkdv_sample_batch): accepted index sets, stored rows
  and statistics for the Sigma and the uniform proposal, accepted-count mode,
  ragged sizes, and a batch mixing K = 32 and K = 128.
The rejection constants come from the library's host search (the oracle's own
Nelder-Mead is too slow at 256 dimensions); both sides take the same plan.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from conftest import check_extremes

pytestmark = pytest.mark.gpu

AMBIG = 1e-9
K = 128
N = 4 * K


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


@pytest.fixture(scope="module")
def case(T):
    """(beta', C3/C2) = (20, 1500): acceptance about 1.4e-2 at K = 128."""
    pt = T.make_point(K, 1.0, 20.0, 1500.0, seed=11, point_id=3)
    say("planning K=128 (host search)")
    return pt, T.plan_point(pt, T.SIGMA)


def oracle_S3(xhat):
    """sum_j u~_j^3 and sum_j |u~_j|^3 on the N = 4K standard grid (E0 = pi/2: u = u~)."""
    s3 = np.empty(xhat.shape[0])
    sa = np.empty(xhat.shape[0])
    for r in range(xhat.shape[0]):
        u = oracle.grid(xhat[r], math.pi / 2, N)
        s3[r] = np.sum(u ** 3)
        sa[r] = np.sum(np.abs(u) ** 3)
    return s3, sa


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_eval_k128_uniform_against_oracle(T, ctx, prec):
    """The uniform proposal (no Sigma scaling of the draw) per proposal at K = 128."""
    pt = T.make_point(K, 1.0, 20.0, 1500.0, seed=13, point_id=5)
    plan = T.plan_point(pt, T.UNIFORM)
    n, i0 = 16 * 9 + 7, 12345
    P = T.PRECISIONS[prec]
    g = {k: v.cpu().numpy() for k, v in ctx.eval_proposals(pt, i0, n, proposal=T.UNIFORM, plan=plan,
                                                            precision=P).items()}
    o = oracle.sample(K, pt.E0, pt.beta_p, pt.c32, 0, plan.alpha_star, plan.log_M, pt.seed, pt.point_id, n, N,
                      i0=i0, cap=0, want_log=True)
    xo = np.stack([oracle.proposal(K, 1.0, pt.beta_p, pt.c32, 0, plan.alpha_star, plan.log_M, pt.seed,
                                   pt.point_id, i0 + q)[0] for q in range(n)])
    dx = np.linalg.norm(g["xhat"].astype(np.float64) - xo, axis=1)
    say(f"uniform K=128 {prec}: max |dx^| = {dx.max():.3e}")
    assert dx.max() < 2e-6
    k2 = (np.arange(1, K + 1) ** 2).astype(np.float64)
    to = (xo[:, :K] ** 2 + xo[:, K:] ** 2) @ k2
    assert np.max(np.abs(g["t"] - to) / to) < 1e-5
    tau = T.decision_window(pt, T.UNIFORM, P)
    err = np.abs(g["log_a"].astype(np.float64) - o["log_a"])
    say(f"   max|dlog a| = {err.max():.3e}, window = {tau:.3e}")
    assert err.max() < tau / 2
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    assert not ((g["accept"].astype(bool) != o["accept"].astype(bool)) & ~amb).any()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("n,i0", [(16 * 67 + 5, 0), (16 * 3 + 9, (1 << 33) + 7)])
def test_eval_k128_against_oracle(T, ctx, case, prec, n, i0):
    pt, plan = case
    say(f"eval K=128 n={n} i0={i0} prec={prec}")
    P = T.PRECISIONS[prec]
    g = {k: v.cpu().numpy() for k, v in ctx.eval_proposals(pt, i0, n, plan=plan, precision=P).items()}
    o = oracle.sample(K, pt.E0, pt.beta_p, pt.c32, 1, plan.alpha_star, plan.log_M, pt.seed, pt.point_id, n, N,
                      i0=i0, cap=0, want_log=True)
    xo = np.stack([oracle.proposal(K, 1.0, pt.beta_p, pt.c32, 1, plan.alpha_star, plan.log_M, pt.seed,
                                   pt.point_id, i0 + q)[0] for q in range(n)])
    dx = np.linalg.norm(g["xhat"].astype(np.float64) - xo, axis=1)
    say(f"   max |dx^| = {dx.max():.3e}")
    assert dx.max() < 2e-6
    k2 = (np.arange(1, K + 1) ** 2).astype(np.float64)
    to = (xo[:, :K] ** 2 + xo[:, K:] ** 2) @ k2
    assert np.max(np.abs(g["t"] - to) / to) < 1e-5
    s3o, sa = oracle_S3(xo)
    eps = {"fp32": 0.0, "bf16x3": 3.02 * 2.0 ** -18}[prec] + K * 2.0 ** -23
    bound = 3 * (N / 2) * np.sqrt(K) * (eps + dx.max()) + N * 2.0 ** -23 * np.sqrt(K) * N / 2
    ds3 = np.abs(g["s3"] - s3o)
    say(f"   max|dS3| = {ds3.max():.3e} (bound {bound:.3e}), max|dS3|/S3abs = {(ds3 / sa).max():.3e}")
    assert ds3.max() < bound
    assert (ds3 / sa).max() < {"fp32": 1e-6, "bf16x3": 1e-5}[prec]
    tau = T.decision_window(pt, T.SIGMA, P)
    err = np.abs(g["log_a"].astype(np.float64) - o["log_a"])
    say(f"   max|dlog a| = {err.max():.3e}, window = {tau:.3e}")
    assert err.max() < tau / 2
    assert np.max(np.abs(g["log_u"] - o["log_u"])) < 1e-6
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    mism = (g["accept"].astype(bool) != o["accept"].astype(bool)) & ~amb
    assert not mism.any(), f"{mism.sum()} decisions differ"


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_k128_H_error_over_2_16_proposals(T, ctx, case, prec):
    """The worst case over 2^16 proposals: H3 against the cube-sum scale (FP32
    1e-6, BF16x3 1e-5) and H = H2 - (C3/C2) H3 relative to itself (1e-6)."""
    pt, plan = case
    n = 1 << 16
    say(f"H error K=128 n={n} prec={prec}")
    o = oracle.eval_batch(K, pt.E0, pt.beta_p, pt.c32, 1, plan.alpha_star, plan.log_M, pt.seed, pt.point_id, 0, n,
                          N)
    g = ctx.eval_proposals(pt, 0, n, plan=plan, precision=T.PRECISIONS[prec])
    s3 = g["s3"].cpu().numpy().astype(np.float64)
    t = g["t"].cpu().numpy().astype(np.float64)
    rel3 = np.abs(s3 - o["S3"]) / o["S3abs"]
    h3_of = math.pi / (3 * N) * (2 * pt.E0 / math.pi) ** 1.5
    H_o = o["H2"] - pt.c32 * h3_of * o["S3"]
    relH = np.abs(pt.E0 * t - pt.c32 * h3_of * s3 - H_o) / np.abs(H_o)
    say(f"   H3 max {rel3.max():.3e} median {np.median(rel3):.3e}; H max {relH.max():.3e}")
    assert rel3.max() < {"fp32": 1e-6, "bf16x3": 1e-5}[prec]
    assert relH.max() < 1e-6


@pytest.mark.parametrize("prop,n,prec", [(1, 150_003, "bf16x3"), (1, 40_017, "fp32"), (0, 50_001, "bf16x3")])
def test_sample_k128_matches_oracle(T, ctx, case, prop, n, prec):
    if prop == 1:
        pt, plan = case
    else:  # the uniform proposal at a point where it accepts often
        pt = T.make_point(K, 1.0, 2.0, 30.0, seed=4, point_id=8)
        plan = T.plan_point(pt, T.UNIFORM)
    say(f"sample K=128 prop={prop} n={n} prec={prec}")
    cap = n
    r = ctx.sample(pt, n, proposal=prop, plan=plan, precision=T.PRECISIONS[prec], capacity=cap)
    o = oracle.sample(K, pt.E0, pt.beta_p, pt.c32, prop, plan.alpha_star, plan.log_M, pt.seed, pt.point_id, n, N,
                      cap=cap, want_log=True)
    amb = np.abs(o["log_u"] - o["log_a"]) < AMBIG
    acc_o = o["accept"].astype(bool)
    idx_g = r["index"].cpu().numpy().astype(np.int64)
    acc_g = np.zeros(n, dtype=bool)
    acc_g[idx_g] = True
    say(f"   accepted gpu={r['n_accepted']} oracle={int(acc_o.sum())} fp64={r['n_fp64_fixups']}")
    assert acc_o.sum() > 50
    assert not ((acc_g != acc_o) & ~amb).any()
    assert r["n_proposed"] == n and r["n_accepted"] == acc_g.sum() == len(idx_g)
    assert np.all(np.diff(idx_g) > 0)
    same = np.isin(idx_g, o["index"])
    xg = r["xhat"].cpu().numpy().astype(np.float64)[same]
    xo = o["xhat"][np.isin(o["index"], idx_g)]
    assert np.max(np.linalg.norm(xg - xo, axis=1)) < 2e-6
    so = o["stats"]
    for name in ("S2", "S4"):
        assert r[name] == pytest.approx(getattr(so, name), rel=2e-5)
    for name in ("S1", "S3"):
        assert abs(r[name] - getattr(so, name)) < 2e-5 * so.S2 ** (1 if name == "S1" else 1.5) + 1e-9
    assert r["n_grid_values"] == so.n_grid
    assert abs(int(r["n_exceed_2sigma"]) - int(so.n_exceed)) <= 2 + so.n_exceed // 100000
    assert np.abs(r["hist_u0"].astype(np.int64) - so.hist.astype(np.int64)).sum() <= 2
    check_extremes(r, so, pt.E0, K, o["xhat"], o["index"])
    assert r["n_M_violations"] == 0


def test_k128_accepted_count_mode_and_ragged_sizes(T, ctx, case):
    pt, plan = case
    target = 300
    say("accepted-count K=128")
    r = ctx.sample(pt, target, plan=plan, mode=T.COUNT_ACCEPTED, max_proposals=2_000_000, capacity=target,
                   precision=T.BF16X3)
    o = oracle.sample_until(K, pt.E0, pt.beta_p, pt.c32, 1, plan.alpha_star, plan.log_M, pt.seed, pt.point_id,
                            target, 2_000_000, N)
    assert r["n_accepted"] == target
    assert np.array_equal(r["index"].cpu().numpy().astype(np.uint64), o["index"])
    assert r["n_proposed"] == o["stats"].n_proposed
    assert r["S2"] == pytest.approx(o["stats"].S2, rel=2e-5)
    # beta' = 0: every proposal accepted; ragged tails of the 16-proposal tiles
    p0 = T.make_point(K, 1.0, 0.0, 0.0, seed=9, point_id=4)
    pl0 = T.plan_point(p0, T.SIGMA)
    for n in (1, 15, 16, 17, 33, 2048 + 1):
        a = ctx.sample(p0, n, plan=pl0, capacity=n)
        b = ctx.sample(p0, n, plan=pl0, capacity=n)
        assert a["n_accepted"] == n
        assert np.array_equal(a["index"].cpu().numpy(), np.arange(n))
        assert np.array_equal(a["xhat"].cpu().numpy(), b["xhat"].cpu().numpy())
        assert a["S2"] / a["n_grid_values"] == pytest.approx(1 / math.pi, rel=1e-6)


def test_k128_in_a_batch_with_k32(T, ctx, case):
    pt, plan = case
    p32 = T.make_point(32, 1.0, 40.0, 75.0, seed=21, point_id=1)
    pl32 = T.plan_point(p32, T.SIGMA)
    pts, plans, ns = [pt, p32], [plan, pl32], [70_001, 40_000]
    caps = [20_000, 20_000]
    out, _, _ = ctx.sample_batch(pts, ns, plans=plans, capacity=caps)
    for p in range(2):
        single = ctx.sample(pts[p], ns[p], plan=plans[p], capacity=caps[p])
        assert out[p]["n_accepted"] == single["n_accepted"]
        assert np.array_equal(out[p]["index"].cpu().numpy(), single["index"].cpu().numpy())
        assert np.array_equal(out[p]["xhat"].cpu().numpy()[:, : 2 * pts[p].K], single["xhat"].cpu().numpy())
        assert out[p]["S3"] == single["S3"]
