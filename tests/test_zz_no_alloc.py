"""tkdv_sample_noalloc, the sampling entry point that allocates nothing, against tkdv_sample.

Through the C ABI, on one context: two calls in a row, the second with a
smaller input, each equal to tkdv_sample's result on the same point (the same
kernels on other buffers: accepted indices, rows and statistics bit for bit),
in proposal-count and accepted-count mode; sizes beyond the fixed scratch and
a missing plan are refused; and a call of 2^25 proposals, whose work buffers
would take 12 MB, leaves the device's free memory unchanged.
"""
import ctypes as C
import sys

import numpy as np
import pytest

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


def _same(ref, got):
    for key in ("n_proposed", "n_accepted", "n_written", "n_fp64_fixups", "n_M_violations", "n_exceed_2sigma",
                "n_grid_values", "S1", "S2", "S3", "S4", "max_log_a", "log_M_used", "M_raises"):
        assert got[key] == ref[key], (key, got[key], ref[key])
    assert np.array_equal(got["hist_u0"], ref["hist_u0"])
    assert np.array_equal(got["index"].cpu().numpy(), ref["index"].cpu().numpy())
    assert np.array_equal(got["xhat"].cpu().numpy(), ref["xhat"].cpu().numpy())


def test_noalloc_equals_sample_on_two_calls_in_a_row(T):
    import torch
    ctx = T.Context(0)
    cap = 40_000
    # the second call is smaller (fewer proposals and another K), so any state the
    # first leaves in the shared array would show
    cases = [(32, 40.0, 75.0, 1_000_003, T.COUNT_PROPOSALS, T.BF16X3),
             (16, 40.0, 60.0, 70_001, T.COUNT_PROPOSALS, T.FP32),
             (8, 40.0, 20.0, 900, T.COUNT_ACCEPTED, T.BF16X3)]
    pts = [T.make_point(K, 1.0, bp, c, seed=3, point_id=7 + q) for q, (K, bp, c, *_r) in enumerate(cases)]
    plans = [T.plan_point(p, T.SIGMA) for p in pts]
    refs = [ctx.sample(p, n, plan=pl, mode=mode, max_proposals=2_000_000, precision=prec, capacity=cap)
            for p, pl, (_, _, _, n, mode, prec) in zip(pts, plans, cases)]
    outs = []
    for p, pl, (K, _, _, n, mode, prec) in zip(pts, plans, cases):
        xh = torch.empty((cap, 2 * K), dtype=torch.float32, device="cuda")
        ix = torch.empty((cap,), dtype=torch.int64, device="cuda")
        outs.append(ctx.sample_noalloc(p, n, pl, mode=mode, max_proposals=2_000_000, precision=prec, xhat=xh,
                                       index=ix))
    for (K, _, _, n, _, _), ref, got in zip(cases, refs, outs):
        say(f"K={K} n={n}: accepted {got['n_accepted']} (tkdv_sample {ref['n_accepted']})")
        assert ref["n_accepted"] > 0
        _same(ref, got)
    ctx.close()


def test_noalloc_limits_and_no_device_memory(T):
    import torch
    ctx = T.Context(0)
    pt = T.make_point(16, 1.0, 40.0, 60.0, seed=1, point_id=2)
    plan = T.plan_point(pt, T.SIGMA)
    xh = torch.empty((1000, 32), dtype=torch.float32, device="cuda")
    ix = torch.empty((1000,), dtype=torch.int64, device="cuda")
    ctx.sample_noalloc(pt, 4096, plan, xhat=xh, index=ix)   # every kernel of the path loaded once
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    r = ctx.sample_noalloc(pt, 1 << 25, plan, xhat=xh, index=ix)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"2^25 proposals: {r['n_accepted']} accepted; free memory {free0} -> {free1}")
    assert r["n_proposed"] == 1 << 25 and r["n_accepted"] > 0
    assert free0 - free1 < (4 << 20)
    with pytest.raises(T.TkdvError) as e:   # beyond the fixed scratch
        ctx.sample_noalloc(pt, (1 << 26) + 1, plan, xhat=xh, index=ix)
    assert e.value.status == -1
    st = T.Stats()                          # the plan is required
    rc = T.lib.tkdv_sample_noalloc(ctx._h, C.byref(pt), T.SIGMA, None, 100, T.COUNT_PROPOSALS, 0, T.BF16X3,
                                   None, None, 0, C.byref(st), None)
    assert rc == -1
    ctx.close()
