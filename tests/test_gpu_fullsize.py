"""Parity at full size, in the benchmark's launch configurations.

The samplers run 1e9 proposals per point (the plain GPU and learned
configurations): the paper's sampler as one batched launch over two K = 32
points, the mixture sampler on one K = 32 point.  The oracle then checks
sampled outputs one by one: 600 random proposal indices over the whole range
(decision and, for accepted ones, the stored row), and 300 random accepted
samples (an accept in FP64, the same row); the accepted count must be
consistent with the acceptance of the random indices.
"""
import math
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

N_PROP = 10**9
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


def _check_sampled(res, decide, n, rng, label):
    """decide(i) -> (x^ [2K], log_a, log_u) from the oracle."""
    idx = res["index"].cpu().numpy().astype(np.int64)
    rows = res["xhat"].cpu().numpy().astype(np.float64)
    assert res["n_written"] == res["n_accepted"], "all accepted samples are stored"
    assert np.all(np.diff(idx) > 0), "rows in increasing proposal index"
    pos = {int(i): r for r, i in enumerate(idx)}
    # random indices over the whole range
    checked = 0
    for i in rng.integers(0, n, 600):
        x, la, lu = decide(int(i))
        if abs(la - lu) < AMBIG:
            continue
        acc = lu < la
        assert (int(i) in pos) == acc, f"{label}: decision of proposal {i} differs"
        if acc:
            assert np.linalg.norm(rows[pos[int(i)]] - x) < 1e-5
        checked += 1
    # random accepted samples
    for r in rng.integers(0, len(idx), 300):
        x, la, lu = decide(int(idx[r]))
        assert lu < la + AMBIG, f"{label}: proposal {idx[r]} accepted on the GPU, rejected in FP64"
        assert np.linalg.norm(rows[r] - x) < 1e-5
    say(f"{label}: {res['n_accepted']} accepted of {n}, {checked} random indices and 300 accepted rows checked")


def test_plain_batch_1e9(T, ctx):
    K = 32
    pts = [T.make_point(K, 1.0, bp, 6000.0 / bp, seed=11 + i, point_id=i) for i, bp in enumerate((30.0, 45.0))]
    plans = [T.plan_point(p, T.SIGMA) for p in pts]
    cap = [1 << 21] * 2
    out, _, _ = ctx.sample_batch(pts, [N_PROP] * 2, plans=plans, precision=T.BF16X3, capacity=cap)
    rng = np.random.default_rng(5)
    for p, pl, o in zip(pts, plans, out):
        assert o["n_proposed"] == N_PROP and o["n_M_violations"] == 0

        def decide(i, p=p, pl=pl):
            x, la, lu = oracle.proposal(K, 1.0, p.beta_p, p.c32, 1, pl.alpha_star, pl.log_M, p.seed, p.point_id, i)
            return x, la, lu

        _check_sampled(o, decide, N_PROP, rng, f"plain beta'={p.beta_p}")
        acc = o["n_accepted"] / N_PROP
        assert 1e-4 < acc < 1e-2


def test_mixture_1e9(T, ctx):
    K, bp, c = 32, 40.0, 225.0
    pt = T.make_point(K, 1.0, bp, c, seed=21, point_id=3)
    sp = T.plan_point(pt, T.SIGMA)
    rng = np.random.default_rng(6)
    logd = np.log(np.array(sp.sigma2[:K])) + 0.1 * rng.standard_normal(K)
    V = 0.8 * rng.standard_normal((2 * K, 2)) / math.sqrt(K)
    mx = T.make_mixture(K, 0.2, logd, V)
    mo = oracle.make_mixture(K, 0.2, logd, V)
    pl, _ = T.plan_mixture(pt, sp, mx, margin=0.02)
    o = ctx.sample_mixture(pt, pl, mx, N_PROP, precision=T.BF16X3, capacity=1 << 22)
    assert o["n_proposed"] == N_PROP and o["n_M_violations"] == 0

    def decide(i):
        return oracle.mix_proposal(K, 1.0, bp, c, pl.alpha_star, pl.log_M, mo, pt.seed, pt.point_id, i)

    _check_sampled(o, decide, N_PROP, rng, "mixture")
