"""Host-side checks of the C ABI (no GPU needed).

The library loads and exports every function declared in include/tkdv.h; the
host plan (alpha*, log M) agrees with the oracle's independent plan; argument
validation returns the documented status codes.
"""
import math
import os
import re

import pytest

import oracle
from oracle import plan as oplan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tkdv.h")).read()
    # declarations: "<type> [*]tkdv_name(" at the start of a line
    return sorted(set(re.findall(r"^[a-z_ ]+\**\s*\*?(tkdv_[a-z_]+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2411_16952_amd import tkdv as T
    declared = header_functions()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(T.lib, name), f"{name} declared in tkdv.h but not exported"
    assert set(declared) == set(T.EXPORTS)


@pytest.mark.parametrize("K,bp,c", [(8, 40.0, 20.0), (16, 20.0, 60.0), (16, 40.0, 0.0), (8, 0.0, 5.0)])
def test_host_plan_matches_oracle(K, bp, c):
    from paper_2411_16952_amd import tkdv as T
    pt = T.make_point(K, 1.0, bp, c)
    for prop in (T.SIGMA, T.UNIFORM):
        pl = T.plan_point(pt, prop)
        op = oplan.plan_point(K, 1.0, bp, c, proposal=prop, n_random=0)
        assert pl.alpha_star == pytest.approx(op.alpha_star, rel=1e-14)
        assert pl.log_M == pytest.approx(op.log_M, abs=1e-9)
        for k in range(K):
            assert pl.sigma2[k] == pytest.approx(op.sigma2[k], rel=1e-14)
        if prop == T.SIGMA:
            lng = sum(math.log1p(pl.alpha_star * bp * (k + 1) ** 2 / K**3) for k in range(K))
            assert pl.log_norm_g == pytest.approx(lng, rel=1e-13, abs=1e-15)
        assert pl.N == 4 * K


def test_plan_argument_errors():
    from paper_2411_16952_amd import tkdv as T
    with pytest.raises(T.TkdvError) as e:
        T.plan_point(T.make_point(8, -1.0, 40.0, 0.0))
    assert e.value.status == -1
    with pytest.raises(T.TkdvError) as e:
        T.plan_point(T.make_point(8, 1.0, -1.0, 0.0))
    assert e.value.status == -1
    with pytest.raises(T.TkdvError) as e:
        T.plan_point(T.make_point(8, 1.0, 40.0, float("nan")))
    assert e.value.status == -1
    with pytest.raises(T.TkdvError) as e:  # beta' beyond K^2 sum 1/k^2: no root of F
        T.plan_point(T.make_point(2, 1.0, 5.0, 0.0))
    assert e.value.status == -2
    with pytest.raises(T.TkdvError) as e:
        T.plan_point(T.make_point(0, 1.0, 1.0, 0.0))
    assert e.value.status == -1


def test_decision_window_orders_precisions():
    """The window bounds the fast path's error: it widens from FP32 to BF16x3
    to BF16 and grows with beta' C3/C2."""
    from paper_2411_16952_amd import tkdv as T
    pt = T.make_point(16, 1.0, 40.0, 60.0)
    w = [T.decision_window(pt, T.SIGMA, p) for p in (T.FP32, T.BF16X3, T.BF16)]
    assert 0 < w[0] < w[1] < w[2] < 1.0
    w2 = T.decision_window(T.make_point(16, 1.0, 40.0, 120.0), T.SIGMA, T.BF16X3)
    assert w2 > w[1]
