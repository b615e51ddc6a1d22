"""Precision of the synthesis arithmetic against the FP64 oracle (K = 64, N = 256).

One batch of 2^20 Sigma proposals at beta' = 40, C3/C2 in {0, 300}: the fast
path's H3 (grid sum of cubes), H2 and H = H2 - (C3/C2) H3 for FP32 and BF16x3
products, compared proposal by proposal with the oracle (H3 relative to the
scale S3abs = sum_j |u_j|^3, H2 and H relative to themselves); accept-decision
mismatches of the FP32 fast path alone and after the FP64 re-decision; and
the standalone synthesis kernel (x^ read from HBM) on the same rows, which
also gives the plain BF16 products' error (no decision is taken with those).
Bounds: FP32 1e-6 and BF16x3 1e-5 on H3 in the worst case, 1e-6 on H; plain
BF16 1e-3 on H, and on H3 1e-3 in the median with its worst case pinned below
4e-3.  A JSON report is
written to the directory named by the environment variable TKDV_REPORT_DIR
when it is set.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

N_BATCH = 1 << 20


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


@pytest.mark.parametrize("c32", [0.0, 300.0])
def test_precision_study_k64(T, ctx, c32):
    K, E0, bp = 64, 1.0, 40.0
    N = 4 * K
    print(f"precision study K={K} beta'={bp} c={c32} n={N_BATCH}", flush=True)
    pt = T.make_point(K, E0, bp, c32, seed=7, point_id=int(c32 > 0))
    plan = T.plan_point(pt, T.SIGMA)
    o = oracle.eval_batch(K, E0, bp, c32, 1, plan.alpha_star, plan.log_M, pt.seed, pt.point_id, 0, N_BATCH, N)
    t_o = o["H2"] / E0
    amb = np.abs(o["log_u"] - o["log_a"]) < 1e-9
    dec_o = o["log_u"] < o["log_a"]
    # H3 = (pi/(3N)) (2 E0/pi)^{3/2} S3 (Sec. II.A on the grid); H/C2 = H2 - (C3/C2) H3
    h3_of = math.pi / (3 * N) * (2 * E0 / math.pi) ** 1.5
    H_o = o["H2"] - c32 * h3_of * o["S3"]
    report = {"K": K, "N": N, "beta_p": bp, "c32": c32, "n": N_BATCH,
              "oracle_accepted": int(dec_o.sum()), "ambiguous": int(amb.sum()), "precisions": {}}
    # worst case of |dH3| against the cube-sum scale (pi/3N) sum_j |u_j|^3 (the
    # scale of H3, which itself can vanish): FP32 1e-6; BF16x3 below the
    # per-product bound 3 2^-18 of its split; the whole H to 1e-6 relative
    bounds = {"fp32": 1e-6, "bf16x3": 1e-5}
    xhat_fp32 = None
    for name in ("fp32", "bf16x3"):
        P = T.PRECISIONS[name]
        g = ctx.eval_proposals(pt, 0, N_BATCH, plan=plan, precision=P)
        s3_sa = ctx.synthesize(g["xhat"], precision=P).cpu().numpy().astype(np.float64)
        s3 = g["s3"].cpu().numpy().astype(np.float64)
        t = g["t"].cpu().numpy().astype(np.float64)
        la = g["log_a"].cpu().numpy().astype(np.float64)
        lu = g["log_u"].cpu().numpy().astype(np.float64)
        acc = g["accept"].cpu().numpy().astype(bool)
        if name == "fp32":
            xhat_fp32, t_fp32 = g["xhat"], t
        del g
        rel3 = np.abs(s3 - o["S3"]) / o["S3abs"]
        rel3_sa = np.abs(s3_sa - o["S3"]) / o["S3abs"]
        rel2 = np.abs(t - t_o) / t_o
        relH = np.abs(E0 * t - c32 * h3_of * s3 - H_o) / np.abs(H_o)
        fast = lu < la
        rep = {
            "H3_rel_max": float(rel3.max()), "H3_rel_median": float(np.median(rel3)),
            "H3_rel_max_standalone": float(rel3_sa.max()),
            "H3_rel_median_standalone": float(np.median(rel3_sa)),
            "H2_rel_max": float(rel2.max()), "H2_rel_median": float(np.median(rel2)),
            "H_rel_max": float(relH.max()), "H_rel_median": float(np.median(relH)),
            "log_a_abs_max": float(np.abs(la - o["log_a"]).max()),
            "window": T.decision_window(pt, T.SIGMA, P),
            "decision_mismatch_fast_path": int(((fast != dec_o) & ~amb).sum()),
            "decision_mismatch_after_fp64": int(((acc != dec_o) & ~amb).sum()),
        }
        report["precisions"][name] = rep
        print(name, json.dumps(rep), flush=True)
        assert rep["decision_mismatch_after_fp64"] == 0
        assert rep["H3_rel_max"] < bounds[name] and rep["H3_rel_max_standalone"] < bounds[name]
        assert rep["H2_rel_max"] < 1e-6
        assert rep["H_rel_max"] < 1e-6
        assert rep["log_a_abs_max"] < rep["window"] / 2
    # plain BF16 products (synthesis only: the library takes no decision with
    # them) on the same FP32 rows; H2 from the FP32 path
    s3_b = ctx.synthesize(xhat_fp32, precision=T.BF16).cpu().numpy().astype(np.float64)
    rel3 = np.abs(s3_b - o["S3"]) / o["S3abs"]
    relH = np.abs(E0 * t_fp32 - c32 * h3_of * s3_b - H_o) / np.abs(H_o)
    rep = {"H3_rel_max_standalone": float(rel3.max()), "H3_rel_median_standalone": float(np.median(rel3)),
           "H_rel_max": float(relH.max()), "H_rel_median": float(np.median(relH))}
    report["precisions"]["bf16"] = rep
    print("bf16", json.dumps(rep), flush=True)
    # the whole H meets 1e-3; H3 on its own scale meets it in the median but
    # not in the worst case (measured 2.9e-3): this pins that miss
    assert rep["H_rel_max"] < 1e-3
    assert rep["H3_rel_median_standalone"] < 1e-3
    assert rep["H3_rel_max_standalone"] < 4e-3
    out = os.environ.get("TKDV_REPORT_DIR", "")
    if out and os.path.isdir(out):
        with open(os.path.join(out, f"precision_k64_c{int(c32)}.json"), "w") as f:
            json.dump(report, f, indent=1)
    sys.stdout.flush()
