"""The batched sweep (tkdv_sample_sweep) and its autotuner on the GPU.

* windows: a sweep over points of every K, with fixed windows much smaller
  than the proposals each point needs and with windows sized on the device
  from the measured acceptance, gives, point by point, the same accepted
  samples (indices and rows, bit for bit), the same proposal count and the
  same statistics as a single accepted-count call of that point; the
  adaptive sweep of these points is one graph launch;
* the hipGraph launch of 16 windows gives bit-identical results to launching
  the same sequence directly, and to itself on a second call;
* every tile variant of the decision kernel gives bit-identical results (at
  K = 16, 32, 64 and, with its workgroup sizes, at K = 128);
* a point that reaches its proposal cap stops there;
* against the oracle: the first n accepted samples of a K = 8, 16, 32, 64
  and 128 point (K = 128 also with its 1024-thread tile variant);
* the autotuner returns a valid configuration (variant, workgroups per
  compute unit, first window) and reads it back from its cache.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from conftest import check_extremes

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


SPECS = [  # K, beta', C3/C2, target, max proposals (acceptance ~3e-3, 3e-2, 3e-2, 0.1, 1e-3, 2e-2)
    (8, 40.0, 20.0, 700, 1 << 26),
    (16, 20.0, 60.0, 10000, 1 << 26),
    (32, 40.0, 75.0, 9000, 1 << 27),
    (64, 40.0, 150.0, 20000, 1 << 26),
    (32, 20.0, 300.0, 5000, 3_000_017),   # cap reached before the target
    (16, 40.0, 30.0, 12000, 1 << 26),
    (128, 40.0, 750.0, 3000, 1 << 24),    # the quarter-period kernels
]


def _points(T):
    pts = [T.make_point(K, 1.0, bp, c, seed=31 + i, point_id=i) for i, (K, bp, c, _, _) in enumerate(SPECS)]
    plans = [T.plan_point(p, T.SIGMA) for p in pts]
    return pts, plans


@pytest.mark.parametrize("use_graph,adaptive", [(0, 0), (1, 0), (1, 1)])
def test_sweep_equals_single_point_calls(T, ctx, use_graph, adaptive):
    pts, plans = _points(T)
    targets = [s[3] for s in SPECS]
    maxp = [s[4] for s in SPECS]
    # first windows of 2^16 proposals: several windows per point
    cfg = T.LaunchCfg(0, use_graph, 1 << 16, 0, adaptive)
    caps = [t + 5 for t in targets]
    out, _, _ = ctx.sample_sweep(pts, targets, maxp, plans=plans, precision=T.BF16X3, cfg=cfg, capacity=caps)
    tm = ctx.timing()
    windows = tm["windows"]
    say(f"use_graph={use_graph} adaptive={adaptive}: {windows} windows, {tm['graph_launches']} launches, "
        f"{tm['total_ms']:.1f} ms")
    for i, o in enumerate(out):
        say(f"   point {i}: accepted {o['n_accepted']} proposed {o['n_proposed']} written {o['n_written']}")
    assert windows > (1 if adaptive else 4)
    if adaptive:
        assert tm["graph_launches"] == 1
    for i, (p, pl, o) in enumerate(zip(pts, plans, out)):
        r = ctx.sample(p, targets[i], proposal=T.SIGMA, plan=pl, mode=T.COUNT_ACCEPTED, max_proposals=maxp[i],
                       precision=T.BF16X3, capacity=caps[i])
        say(f"point {i} K={p.K}: sweep acc {o['n_accepted']} prop {o['n_proposed']}; "
            f"single acc {r['n_accepted']} prop {r['n_proposed']}")
        assert o["n_accepted"] == r["n_accepted"] and o["n_proposed"] == r["n_proposed"]
        assert o["n_written"] == r["n_written"]
        assert np.array_equal(o["index"].cpu().numpy(), r["index"].cpu().numpy())
        assert np.array_equal(o["xhat"].cpu().numpy(), r["xhat"].cpu().numpy())
        assert o["hist_u0"].tolist() == r["hist_u0"].tolist()
        assert o["n_exceed_2sigma"] == r["n_exceed_2sigma"]
        for f in ("n_exceed_4sigma", "n_samples_4sigma", "peak_u", "peak_index"):
            assert o[f] == r[f], f
        for k in ("S1", "S2", "S3", "S4"):  # sums of the same values in another order
            assert abs(o[k] - r[k]) <= 1e-10 * (abs(r[k]) + r["S2"] + 1.0), k
    # the capped point
    assert out[4]["n_accepted"] < targets[4] and out[4]["n_proposed"] == maxp[4]


def test_sweep_graph_replay_is_deterministic(T, ctx):
    pts, plans = _points(T)
    targets = [s[3] for s in SPECS]
    maxp = [s[4] for s in SPECS]
    caps = [t for t in targets]
    res = []
    for use_graph in (1, 0, 1):
        out, _, _ = ctx.sample_sweep(pts, targets, maxp, plans=plans, precision=T.FP32,
                                     cfg=T.LaunchCfg(2, use_graph, 1 << 17), capacity=caps)
        res.append([(o["n_accepted"], o["n_proposed"], o["S3"], o["index"].cpu().numpy().tobytes(),
                     o["xhat"].cpu().numpy().tobytes()) for o in out])
    assert res[0] == res[1] == res[2]


def test_sweep_tile_variants_are_bit_identical(T, ctx):
    """The tuner's variants change the workgroup size and how many tile pairs
    keep their accumulators live together, not the arithmetic."""
    pts, plans = _points(T)
    idx = [1, 2, 3]   # K = 16, 32, 64
    targets = [SPECS[i][3] for i in idx]
    maxp = [SPECS[i][4] for i in idx]
    res = []
    for v in range(4):
        out, _, _ = ctx.sample_sweep([pts[i] for i in idx], targets, maxp, plans=[plans[i] for i in idx],
                                     precision=T.BF16X3, cfg=T.LaunchCfg(0, 1, 1 << 20, v, 1), capacity=targets)
        say(f"variant {v}: {[o['n_accepted'] for o in out]}")
        res.append([(o["n_accepted"], o["n_proposed"], o["S3"], o["index"].cpu().numpy().tobytes(),
                     o["xhat"].cpu().numpy().tobytes()) for o in out])
    assert res[0] == res[1] == res[2] == res[3]


def test_k128_tile_variants_are_bit_identical(T, ctx):
    """At K = 128 the variants are the decision kernel's workgroup sizes
    (768, 512 and 1024 threads: 3, 2 and 4 waves per SIMD)."""
    pts, plans = _points(T)
    i = 6
    res = []
    for v in range(3):
        out, _, _ = ctx.sample_sweep([pts[i]], [SPECS[i][3]], [SPECS[i][4]], plans=[plans[i]], precision=T.BF16X3,
                                     cfg=T.LaunchCfg(0, 1, 1 << 20, v, 1), capacity=[SPECS[i][3]])
        say(f"K=128 variant {v} (block {ctx.timing()['decide_block']}): {out[0]['n_accepted']}")
        res.append((out[0]["n_accepted"], out[0]["n_proposed"], out[0]["S3"], out[0]["index"].cpu().numpy().tobytes(),
                    out[0]["xhat"].cpu().numpy().tobytes()))
    assert res[0] == res[1] == res[2]


@pytest.mark.parametrize("K,bp,c,target,variant", [(8, 40.0, 20.0, 400, 0), (16, 20.0, 60.0, 500, 0),
                                                   (32, 40.0, 75.0, 400, 0), (64, 40.0, 150.0, 300, 0),
                                                   (64, 40.0, 300.0, 300, 3), (128, 40.0, 750.0, 300, 0),
                                                   (128, 40.0, 750.0, 200, 2)])
def test_sweep_against_oracle(T, ctx, K, bp, c, target, variant):
    pt = T.make_point(K, 1.0, bp, c, seed=0, point_id=0)
    pl = T.plan_point(pt, T.SIGMA)
    out, _, _ = ctx.sample_sweep([pt], [target], [1 << 26], plans=[pl], precision=T.BF16X3,
                                 cfg=T.LaunchCfg(0, 1, 1 << 16, variant, 1), capacity=[target])
    say(f"K={K}: {ctx.timing()['windows']} windows")
    o = oracle.sample_until(K, 1.0, bp, c, 1, pl.alpha_star, pl.log_M, 0, 0, target, 1 << 26, 4 * K)
    assert out[0]["n_accepted"] == target == o["stats"].n_accepted
    assert np.array_equal(out[0]["index"].cpu().numpy().astype(np.uint64), o["index"])
    assert out[0]["n_proposed"] == o["stats"].n_proposed
    xg = out[0]["xhat"].cpu().numpy().astype(np.float64)
    assert np.max(np.linalg.norm(xg - o["xhat"], axis=1)) < 2e-6
    assert abs(out[0]["S2"] - o["stats"].S2) < 1e-6 * o["stats"].S2
    assert abs(out[0]["S4"] - o["stats"].S4) < 2e-5 * o["stats"].S4
    check_extremes(out[0], o["stats"], 1.0, K, o["xhat"], o["index"])


def test_sweep_argument_errors(T, ctx):
    pts, plans = _points(T)
    with pytest.raises(T.TkdvError):
        ctx.sample_sweep(pts[:1], [10], [1 << 20], plans=plans[:1], cfg=T.LaunchCfg(0, 1, 1000))  # window
    with pytest.raises(T.TkdvError):
        ctx.sample_sweep(pts[:1], [10], [1 << 20], plans=plans[:1], cfg=T.LaunchCfg(0, 1, 1 << 16, 4))  # variant
    with pytest.raises(T.TkdvError):
        ctx.sample_sweep(pts[:1], [0], [1 << 20], plans=plans[:1])                                # target 0
    up = T.plan_point(pts[0], T.UNIFORM)
    with pytest.raises(T.TkdvError):
        ctx.sample_sweep(pts[:1], [10], [1 << 20], plans=[up])                                    # not Sigma


def test_autotune_and_cache(T, ctx, tmp_path):
    path = str(tmp_path / "tune.txt")
    c1 = ctx.autotune(16, T.BF16X3, path)
    say(f"autotuned K=16: {c1.to_dict()}")
    assert c1.window in (1 << 24, 1 << 25, 1 << 26) and c1.blocks_per_cu >= 1 and c1.use_graph == 1
    assert 0 <= c1.variant < 4 and c1.adaptive == 1
    assert os.path.exists(path) and "K=16" in open(path).read()
    ctx.set_launch_cfg(16, T.BF16X3, T.LaunchCfg(0, 1, 1 << 16))
    c2 = ctx.autotune(16, T.BF16X3, path)      # from the cache
    assert c2.to_dict() == c1.to_dict() == ctx.get_launch_cfg(16, T.BF16X3).to_dict()
    pts, plans = _points(T)
    out, _, _ = ctx.sample_sweep([pts[1]], [200], [1 << 26], plans=[plans[1]], precision=T.BF16X3)
    assert out[0]["n_accepted"] == 200
