#!/usr/bin/env python3
"""Throughput of the MI355X TKdV rejection sampler (arXiv 2411.16952).

Default workload (--workload learned): accepted samples/s at K = 32 with the
learned defensive-mixture proposal against the paper's Sigma proposal.
  * before the timed region: 24 networks (3 -> 256 -> 256 -> 5K, FP64 on
    the GPU, initialisation seeds 1..24) are fitted on 16 training points
    (beta' = linspace(20, 60, 16), C3/C2 = 9000/beta') from the paper's
    sampler's accepted samples, and the plans of the evaluation points are
    made: alpha*, M_Sigma (the paper's step 1) and M_mix of every network's
    mixture (multi-start L-BFGS of f/q_mix on the GPU); each point samples
    with the network whose M_mix there is smallest (acceptance is Z/M_mix);
  * one step: 32 evaluation points (the 16 beta' at beta' C3/C2 = 9000 and
    12000, seeds not used in training), 1e9 proposals per point with the
    mixture sampler, then 1e9 per point with the paper's sampler (one batched
    call), all statistics reduced and up to 2^20 samples per point stored.
  value = the mixture sampler's accepted samples/s; the paper's sampler's
  rate on the same points is reported beside it.  Both samplers are exact,
  so equal accepted counts give equal statistical (KS) accuracy; two-sample
  KS p-values of u(0) between the two samplers' outputs are reported.
--workload plain: the paper's sampler alone on 8 beta' x beta'C3/C2 in
{6000, 12000}, 1e9 proposals per point (the plain GPU configuration).
--workload sweep: 256 points of K in {16, 32, 64} with accepted targets in
[1e4, 1e6] (the batched-sweep configuration), windows replayed as a hipGraph
with the autotuner's launch configuration.
--workload sir: sampling-importance resampling at one K = 32 point (effective
samples/s), beside the rejection sampler and the extreme-wave search.
--workload k128: the paper's sampler at K = 128 (N = 512; the mode count of
its parallel speed-up study), 4 points x 1e9 proposals, quarter-period
synthesis; --workload k64 the same at K = 64 (N = 256).
--synthesis: the standalone synthesis on the precision configuration (K = 64,
2^20 rows of x^ in HBM; HBM roofline), plus the same synthesis with x^ drawn
in registers (the decision kernel).

Prints one JSON line with the roofline of the dominant kernel (ALU-bound:
method-level issue slots, method_ops_per_proposal) from HIP events recorded
inside the library on the kernel's own stream, and the CPU FP64 oracle's
throughput on a bounded sample of the same workload (all host threads, and
one thread).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X vector ALU issue peak: 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3e12 lane-operations/s for instructions without a packed form (a wave
# of 64 lanes issues over 4 clocks; FP64 FMA runs at this rate: 78.6 TFLOP/s).
# The published FP32 vector rate of 157.3 TFLOP/s is twice this with an FMA
# counted as one operation, reached only by packed two-wide FP32 instructions;
# the sampler's operations are mostly integer products, bit operations,
# conversions and transcendentals (quarter rate), which have no packed form,
# and the library is built without packed FP32.  Both figures are reported.
ALU_OPS_PER_S = 256 * 4 * 16 * 2.4e9
PACKED_FP32_OPS_PER_S = 2 * ALU_OPS_PER_S
# HBM3E bandwidth of one MI355X
HBM_BYTES_PER_S = 8.0e12


def dtype_label(precision: str) -> str:
    """Arithmetic of the sampling path: the synthesis products, FP32 for the
    rest of each proposal, FP64 for the re-decision near the threshold and for
    the moment sums."""
    return {"bf16x3": "bf16x3 synthesis + f32 + f64 re-decision",
            "fp32": "f32 synthesis + f32 + f64 re-decision"}[precision]


def alu_roof(achieved: float, **extra) -> dict:
    """Roofline object of an ALU-bound kernel (achieved in lane-operations/s)."""
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_OPS_PER_S / 1e12, "unit": "T ALU ops/s",
         "frac": achieved / ALU_OPS_PER_S}
    r.update(extra)
    r["peak_packed_fp32"] = PACKED_FP32_OPS_PER_S / 1e12
    r["frac_of_packed_fp32"] = achieved / PACKED_FP32_OPS_PER_S
    return r


def method_ops_per_proposal(K: int, proposal: str = "sigma", precision: str = "bf16x3") -> float:
    """Vector-ALU operations one proposal of the method needs, counted once
    and kept fixed: the yardstick of the ALU roofline does not move when a
    kernel finds a cheaper route to the same result (the half- and
    quarter-period syntheses, tables scaled by sqrt 3, the folded Cholesky
    factor: their gain shows as a higher fraction).  Each operation is priced
    at the gfx950 instructions that carry it in the plain form of the method
    (a 32x32 -> 64-bit product, a three-input XOR, an FMA: one issue slot
    each; a transcendental -- log2, exp2, sqrt, 1/sqrt, sin, cos -- one issue
    slot, its execution overlapping the vector ALU):
      Philox4x32-10: K/2 + 1 blocks x 10 rounds x (2 products + 2 three-input XORs)  = 40 (K/2 + 1)
      word -> uniform (2K + 1 words, convert + scale)                               = 2 (2K + 1)
      Box-Muller: K pairs x (log2, sqrt, sin, cos; log scale, 2 products)           = 7 K
      Sigma scaling (2K products; uniform proposal: none)                           = 2 K
      |x|^2 and t = sum k^2 s_k (square, add, FMA per coordinate), lane sums,
        1/sqrt, t scaling                                                           = 6 K + 7
      BF16x3 operands (per coordinate: round, subtract, round)                      = 6 K
      sum of cubes over the N = 4K grid values of the plain synthesis (u u, then
        s += u u^2 per value)                                                       = 8 K
      lane sum and scaling of S3, log a (with log1p), log U, exp2, window edges,
        comparisons                                                                 = 24
    The synthesis products run on the matrix cores (method_mfma_flops).  The
    learned mixture adds, per proposal: component choice from one word (6);
    the Box-Muller pair eta (9); the low-rank part of the draw (4K); Q = X^T A X
    (2K); per shift j < S = 32 the 2x2 quadratic form y^T G^-1 y (5), r_j (1),
    log2, running minimum, exp2 and its sum (4): 10 S; the final log-sum and the
    two-term mixture (20).  At K = 32 with BF16x3: 1769 (Sigma), 2316 (mixture)."""
    split = {"bf16x3": 6 * K, "fp32": 0}[precision]
    scale = 2 * K if proposal in ("sigma", "mixture") else 0
    base = 40 * (K / 2 + 1) + 2 * (2 * K + 1) + 7 * K + scale + 6 * K + 7 + split + 8 * K + 24
    if proposal == "mixture":
        base += 6 + 9 + 4 * K + 2 * K + 10 * 32 + 20
    return base


def method_mfma_flops(K: int, precision: str = "bf16x3", proposal: str = "sigma") -> float:
    """Matrix flops of the method per proposal: the plain synthesis product
    (2K x N with N = 4K, 2 flops per product, per product term: three for
    BF16x3); the mixture adds y = (R_j A V)^T x for 32 shifts x rank 2 rows."""
    rows = 4 * K + (64 if proposal == "mixture" else 0)
    return {"bf16x3": 3, "fp32": 1}[precision] * 2 * (2 * K) * rows


def executed_mfma_flops(K: int, precision: str = "bf16x3", proposal: str = "sigma") -> float:
    """Matrix flops the kernels execute per proposal: K = 8 the plain product;
    K = 16, 32 the half-period form (even and odd modes on half the grid: half
    the plain product); K = 64, 128 the quarter-period form (cos/sin blocks and
    mode parities on a quarter of the offset grid: a quarter); the mixture's y
    products in full."""
    frac = 1.0 if K == 8 else (0.5 if K <= 32 else 0.25)
    terms = {"bf16x3": 3, "fp32": 1}[precision]
    y = 2 * (2 * K) * 64 if proposal == "mixture" else 0
    return terms * (frac * 2 * (2 * K) * (4 * K) + y)


def mfma_peak(precision: str) -> float:
    """Dense matrix peak of MI355X for the products' type (flop/s)."""
    return 157.3e12 if precision == "fp32" else 2.5e15


def mfma_fields(K: int, precision: str, proposal: str, proposals_per_s: float) -> dict:
    ex, me = executed_mfma_flops(K, precision, proposal), method_mfma_flops(K, precision, proposal)
    pk = mfma_peak(precision)
    return {"mfma_flops_executed_per_proposal": ex, "mfma_flops_method_per_proposal": me,
            "mfma_frac_executed": ex * proposals_per_s / pk, "mfma_frac_method": me * proposals_per_s / pk}


def kernel_source_digest(files=("tkdv_device.h", "tkdv_kernels.hip")) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2411_16952_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SYNTH_SOURCES = ("tkdv_device.h", "tkdv_synth.hip")
QUARTER_SOURCES = ("tkdv_device.h", "tkdv_quarter.h", "tkdv_quarter.hip")


def load_traffic(K: int, precision: str, proposals_per_launch: int, kernel: str = "k_decide"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (bytes per proposal, FETCH_SIZE and WRITE_SIZE scaled by the
    plain-copy calibration, times the proposals of this launch), or None when
    the summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_k{K}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src = QUARTER_SOURCES if kernel == "k_decide128" else ("tkdv_device.h", "tkdv_kernels.hip")
    if d.get("kernel_source_digest") != kernel_source_digest(src):
        return None
    return d["bytes_per_proposal"] * proposals_per_launch


def cpu_baseline(points, plans, n_sample: int) -> dict:
    import oracle
    cores = oracle.max_threads()

    def run(n, threads):
        t0 = time.perf_counter()
        n_acc = 0
        for p, pl in zip(points, plans):
            r = oracle.sample(p.K, p.E0, p.beta_p, p.c32, 1, pl.alpha_star, pl.log_M, p.seed, p.point_id,
                              n, 4 * p.K, cap=0, nthreads=threads)
            n_acc += r["stats"].n_accepted
        return n_acc, time.perf_counter() - t0

    n_acc, dt = run(n_sample, cores)
    n_one = max(n_sample // cores, 4096)
    acc1, dt1 = run(n_one, 1)
    n_prop = n_sample * len(points)
    return {
        "value": n_acc / dt, "unit": "accepted samples/s", "cores": cores, "kind": "oracle",
        "context": "the paper reports its CPU sampler at 80% of optimal speedup on 16 cores of an Apple M2 Ultra, K = 128, and gives no absolute rate (Sec. V.C, Fig. 5)",
        "proposals_per_s": n_prop / dt, "accepted": n_acc, "seconds": dt,
        "sample": f"first {n_sample} proposal indices of each of the {len(points)} points "
                  f"({n_prop} proposals, same Philox counters), FP64 oracle with OpenMP",
        "single_core": {"value": acc1 / dt1, "proposals_per_s": n_one * len(points) / dt1, "accepted": acc1,
                        "seconds": dt1, "sample": f"first {n_one} proposal indices of each point, one thread"},
    }


def synthesis_bench(args) -> int:
    """The standalone synthesis u~ = Phi^T x^ plus sum of cubes on the precision
    configuration (2^20 rows, K = 64, N = 256), x^ read from HBM.

    Per row: 8K + 4 bytes of HBM traffic (x^ in, S3 out).  Matrix work: the
    dense product is 2 * 2K * N flops per product term (BF16x3: three terms);
    the kernel executes half of it (even/odd modes with the half-period
    symmetry, K >= 16).  Both fractions are reported; value = rows/s."""
    import torch
    from paper_2411_16952_amd import tkdv as T
    K, n = 64, 1 << 20
    ctx = T.Context(0)
    pt = T.make_point(K, 1.0, 40.0, 300.0, seed=7, point_id=1)
    plan = T.plan_point(pt, T.SIGMA)
    xhat = ctx.eval_proposals(pt, 0, n, plan=plan, precision=T.BF16X3)["xhat"]
    s3 = torch.empty((n,), dtype=torch.float32, device=xhat.device)
    res = {}
    for name in ("bf16x3", "bf16", "fp32"):
        P = T.PRECISIONS[name]
        for _ in range(max(args.warmup, 1)):
            ctx.synthesize(xhat, precision=P, s3=s3)
        ms = []
        for _ in range(max(args.steps, 3)):
            ctx.synthesize(xhat, precision=P, s3=s3)
            ms.append(ctx.timing()["synth_ms"])
        avg = sum(ms) / len(ms)
        dense = {"bf16x3": 3, "bf16": 1, "fp32": 1}[name] * 2.0 * (2 * K) * (4 * K) * n
        executed = dense / 2
        peak = 157.3e12 if name == "fp32" else 2.5e15
        bytes_ = n * (8 * K + 4)
        sec = avg * 1e-3
        res[name] = {"ms": avg, "rows_per_s": n / sec, "hbm_GBps": bytes_ / sec / 1e9,
                     "hbm_frac": bytes_ / sec / HBM_BYTES_PER_S,
                     "mfma_frac_executed": executed / sec / peak, "mfma_frac_method": dense / sec / peak,
                     "grid": ctx.timing()["decide_grid"], "block": ctx.timing()["decide_block"]}
        print(f"synthesis {name}: {avg:.4f} ms", file=sys.stderr, flush=True)
    # the same synthesis with x^ drawn in registers instead of read (Philox, Box-Muller, Sigma
    # scaling): the sampler's decision kernel at this point (the quarter-period form, a quarter
    # of the dense product's matrix work), no samples stored
    n_gen = 16 * n
    gen_ms = []
    for rep in range(1 + max(args.steps, 3)):
        ctx.sample(pt, n_gen, plan=plan, precision=T.BF16X3)
        if rep:
            gen_ms.append(ctx.timing()["decide_ms"])
    g_ms = sum(gen_ms) / len(gen_ms)
    res["bf16x3_from_philox"] = {
        "ms": g_ms, "proposals": n_gen, "rows_per_s": n_gen / (g_ms * 1e-3),
        **mfma_fields(K, "bf16x3", "sigma", n_gen / (g_ms * 1e-3)),
        "alu_frac": method_ops_per_proposal(K) * n_gen / (g_ms * 1e-3) / ALU_OPS_PER_S,
        "kernel": "k_decide128<64> (quarter-period synthesis, decisions included)"}
    print(f"synthesis from Philox (k_decide128<64>, {n_gen} proposals): {g_ms:.3f} ms", file=sys.stderr, flush=True)
    r = res["bf16x3"]
    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated), if taken on these sources
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "k_synth_k64_bf16x3_traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            t = json.load(f)
        if t.get("kernel_source_digest") == kernel_source_digest(SYNTH_SOURCES) and t.get("rows") == n:
            traffic = t["bytes_per_launch"]
    line = {"metric": "synthesis throughput (sum of cubes on the grid, BF16x3 products)", "value": r["rows_per_s"],
            "unit": "rows of x^/s", "higher_is_better": True, "n_gpus": 1, "dtype": "bf16x3",
            "roofline": {"bound": "hbm", "achieved": r["hbm_GBps"], "peak": HBM_BYTES_PER_S / 1e9, "unit": "GB/s",
                         "frac": r["hbm_frac"], "traffic": traffic},
            "config": {"workload": "K=64, N=256, 2^20 rows of x^ (Sigma proposals, beta'=40, C3/C2=300) in HBM",
                       "rows": n, "K": K, "N": 4 * K}, "precisions": res}
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def sir_bench(args) -> int:
    """Sampling-importance resampling (tkdv_sir) on one K = 32 point of the plain
    configuration (beta' = 40, beta'C3/C2 = 6000), beside the rejection
    sampler on the same proposals.  value = effective samples/s (ESS per
    second of the whole call: weights, scan and m = 1e6 draws with rows)."""
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        return 1
    from paper_2411_16952_amd import tkdv as T
    K, bp, c = 32, 40.0, 150.0
    n, m = int(args.proposals), 1_000_000
    prec = T.PRECISIONS[args.precision]
    pt = T.make_point(K, 1.0, bp, c, seed=1, point_id=7)
    pl = T.plan_point(pt, T.SIGMA)
    ctx = T.Context(0)
    for _ in range(args.warmup):
        ctx.sir(pt, n, m, 0.5, plan=pl, precision=prec, rows=True)
    torch.cuda.synchronize()
    wms, tms, ess = [], [], []
    t0 = time.perf_counter()
    for s in range(args.steps):
        r = ctx.sir(pt, n, m, 0.5 + 0.1 * s, plan=pl, precision=prec, rows=True)
        tm = ctx.timing()
        wms.append(tm["decide_ms"])
        tms.append(tm["total_ms"])
        ess.append(r["ess"])
        print(f"sir step {s}: {tm['total_ms']:.1f} ms (weights {tm['decide_ms']:.1f} ms), W {r['W']:.6g}, "
              f"ESS {r['ess']:.6g}, skewness {r['skewness']:.5f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the rejection sampler on the same proposals
    rj = ctx.sample(pt, n, proposal=T.SIGMA, plan=pl, precision=prec, capacity=1 << 20)
    rj_ms = ctx.timing()["total_ms"]
    # the extreme-wave search over the m drawn rows, and GPU plans of 64 points
    rows = r["xhat"]
    ctx.extremes(rows, K, top_k=100)
    torch.cuda.synchronize()
    te = time.perf_counter()
    ex = ctx.extremes(rows, K, top_k=100)
    ext_ms = (time.perf_counter() - te) * 1e3
    pts64 = [T.make_point(K, 1.0, 20.0 + 0.5 * q, 3000.0 / (20.0 + 0.5 * q), seed=q, point_id=q) for q in range(64)]
    ctx.plan_batch(pts64[:2], n_starts=16)
    tp = time.perf_counter()
    ctx.plan_batch(pts64, n_starts=16)
    plan_ms = (time.perf_counter() - tp) * 1e3
    print(f"extremes over {rows.shape[0]} rows: {ext_ms:.2f} ms (largest u {ex['umax'][0]:.4f}, "
          f"{ex['n_exceed']} above 4 sigma); GPU plans of 64 points x 16 starts: {plan_ms:.1f} ms",
          file=sys.stderr, flush=True)
    avg_w = sum(wms) / len(wms) / 1e3
    # the power sums read the plain tables (4 per pair for the cubes), + S1, S2, S4
    # the power sums S1, S2, S4 beside the cubes: 3 more per grid value
    ops = method_ops_per_proposal(K, "sigma", args.precision) + 12 * K
    roof = alu_roof(ops * n / avg_w, traffic=None, kernel="k_sir_weights", method_ops_per_proposal=ops,
                    avg_launch_ms=avg_w * 1e3, proposals_per_launch=n,
                    note="4 B written per proposal (the weights) + 8 B per tile (tile sums)")
    line = {"metric": "effective samples/sec (SIR, K=32)", "value": sum(ess) / dt, "unit": "effective samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(args.precision),
            "data": "synthetic",
            "config": {"workload": f"SIR over {n:.3g} Sigma proposals of K=32, beta'=40, C3/C2={c}, "
                                   f"{m} systematic draws with rows", "K": K, "proposals": n, "draws": m,
                       "synthesis": args.precision},
            "proposals_per_s": n * args.steps / dt, "ess_per_step": sum(ess) / len(ess),
            "rejection": {"accepted": rj["n_accepted"], "ms": rj_ms,
                          "accepted_per_s": rj["n_accepted"] / (rj_ms * 1e-3)},
            "extremes": {"rows": int(rows.shape[0]), "ms": ext_ms, "largest_u": float(ex["umax"][0]),
                         "above_4sigma": ex["n_exceed"]},
            "plan_batch_64_points_16_starts_ms": plan_ms,
            "roofline": roof, "cpu_baseline": None}
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def plain_bench(args) -> int:
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        return 1
    from paper_2411_16952_amd import tkdv as T
    from paper_2411_16952_amd import workloads as W

    specs = W.plain_gpu_points()
    pts = [T.make_point(s.K, s.E0, s.beta_p, s.c32, seed=s.seed, point_id=s.point_id) for s in specs]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=min(16, len(pts))) as ex:
        plans = list(ex.map(lambda p: T.plan_point(p, T.SIGMA), pts))
    plan_s = time.perf_counter() - t0
    K = specs[0].K
    n_per = int(args.proposals)
    n = [n_per] * len(pts)
    cap = [1 << 21] * len(pts)  # every accepted sample of the beta' C3/C2 = 6000 points fits
    prec = T.PRECISIONS[args.precision]
    ctx = T.Context(0)
    print(f"bench: {len(pts)} points, K={K}, {n_per:.3g} proposals/point, {args.precision}, "
          f"plans {plan_s:.2f}s", file=sys.stderr, flush=True)

    def step():
        out, _, _ = ctx.sample_batch(pts, n, plans=plans, precision=prec, capacity=cap)
        return out, ctx.timing()

    for w in range(args.warmup):
        out, tm = step()
        print(f"warmup {w}: {tm['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc, decide_ms, phases = 0, [], []
    t0 = time.perf_counter()
    for s in range(args.steps):
        out, tm = step()
        acc += sum(int(o["n_accepted"]) for o in out)
        decide_ms.append(tm["decide_ms"] / max(tm["decide_launches"], 1))
        phases.append(tm)
        print(f"step {s}: {tm['total_ms']:.1f} ms, decide {tm['decide_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_prop = n_per * len(pts) * args.steps
    fix = sum(int(o["n_fp64_fixups"]) for o in out)
    viol = sum(int(o["n_M_violations"]) for o in out)

    avg_decide_s = sum(decide_ms) / len(decide_ms) / 1e3
    per_launch_props = n_per * len(pts)
    ops = method_ops_per_proposal(K, "sigma", args.precision)
    achieved = ops * per_launch_props / avg_decide_s
    traffic = load_traffic(K, args.precision, per_launch_props)
    roof = alu_roof(achieved, traffic=traffic, kernel="k_decide",
                    method_ops_per_proposal=ops,
                    avg_launch_ms=avg_decide_s * 1e3,
                    proposals_per_launch=per_launch_props,
                    **mfma_fields(K, args.precision, "sigma", per_launch_props / avg_decide_s))

    cpu = None
    n_cpu = (1 << 22) if args.cpu_sample < 0 else args.cpu_sample
    if n_cpu > 0:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(specs, plans, n_cpu)

    line = {
        "metric": "accepted samples/sec at K=32 (plain Sigma proposal); proposals/sec",
        "value": acc / dt,
        "unit": "accepted samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_label(args.precision),
        "data": "synthetic",
        "config": {
            "workload": "plain GPU sweep: K=32, N=128, E0=1, Sigma proposal, beta' in "
                        "{20,25,30,35,40,45,50,60} x beta'C3/C2 in {6000,12000}, 1e9 proposals/point",
            "K": K, "N": 4 * K, "points": len(pts), "proposals_per_point": n_per,
            "synthesis": args.precision, "fp64_redecision": True,
        },
        "proposals_per_s": n_prop / dt,
        "acceptance": acc / n_prop,
        "fp64_redecisions_last_step": fix,
        "M_violations_last_step": viol,
        "plan_seconds": plan_s,
        "phase_ms_last_step": {k: round(v, 3) for k, v in phases[-1].items() if k.endswith("_ms")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0



def cpu_baseline_mixture(points, mixtures, mix_plans, n_sample: int) -> dict:
    """The oracle's mixture sampler (same trained mixtures and M_mix, same
    Philox counters) on the first n_sample proposal indices of every point."""
    import numpy as np
    import oracle
    cores = oracle.max_threads()
    mos = [oracle.make_mixture(p.K, mix.eps, np.array(mix.logd[:p.K]),
                               np.array([[mix.V[r][q] for q in range(2)] for r in range(2 * p.K)]))
           for p, mix in zip(points, mixtures)]

    def run(n, threads):
        t0 = time.perf_counter()
        n_acc = 0
        for p, mo, pl in zip(points, mos, mix_plans):
            r = oracle.mix_sample(p.K, p.E0, p.beta_p, p.c32, pl.alpha_star, pl.log_M, mo, p.seed, p.point_id,
                                  n, nthreads=threads)
            n_acc += int(r["n_accepted"])
        return n_acc, time.perf_counter() - t0

    n_acc, dt = run(n_sample, cores)
    n_one = max(n_sample // cores, 1024)
    acc1, dt1 = run(n_one, 1)
    n_prop = n_sample * len(points)
    return {
        "value": n_acc / dt, "unit": "accepted samples/s", "cores": cores, "kind": "oracle",
        "context": "the paper reports its CPU sampler at 80% of optimal speedup on 16 cores of an Apple M2 Ultra, K = 128, and gives no absolute rate (Sec. V.C, Fig. 5)",
        "proposals_per_s": n_prop / dt, "accepted": n_acc, "seconds": dt,
        "sample": f"first {n_sample} proposal indices of each of the {len(points)} evaluation points "
                  f"({n_prop} proposals, same Philox counters, trained mixtures and M_mix), FP64 oracle "
                  f"mixture sampler with OpenMP",
        "single_core": {"value": acc1 / dt1, "proposals_per_s": n_one * len(points) / dt1, "accepted": acc1,
                        "seconds": dt1, "sample": f"first {n_one} proposal indices of each point, one thread"},
    }


QUARTER_WORKLOADS = {
    "k64": (64, "K=64, N=256, E0=1, Sigma proposal, beta' in {20,40} x beta'C3/C2 in {9000,15000}, "
                "1e9 proposals/point (the mode count of the precision configuration)"),
    "k128": (128, "K=128, N=512, E0=1, Sigma proposal, beta' in {20,40} x beta'C3/C2 in {30000,40000}, "
                  "1e9 proposals/point (the mode count of the paper's speed-up study)"),
}


def quarter_bench(args) -> int:
    """K = 64 (N = 256) or K = 128 (N = 512): the paper's Sigma sampler on 4
    points, 1e9 proposals per point in one batched call (the quarter-period
    decision kernel k_decide128<K>), all statistics and up to 2^20 samples per
    point stored.  value = accepted samples/s; the roofline is the decision
    kernel's launch."""
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        return 1
    from paper_2411_16952_amd import tkdv as T
    from paper_2411_16952_amd import workloads as W

    K, workload = QUARTER_WORKLOADS[args.workload]
    specs = W.k64_points() if K == 64 else W.k128_points()
    pts = [T.make_point(s.K, s.E0, s.beta_p, s.c32, seed=s.seed, point_id=s.point_id) for s in specs]
    ctx = T.Context(0)
    t0 = time.perf_counter()
    plans, _ = ctx.plan_batch(pts, T.SIGMA, n_starts=16, seed=2024)   # log M searched on the GPU
    plan_s = time.perf_counter() - t0
    n_per = int(args.proposals)
    n = [n_per] * len(pts)
    cap = [1 << 20] * len(pts)
    prec = T.PRECISIONS[args.precision]
    print(f"bench: K={K}, {len(pts)} points, {n_per:.3g} proposals/point, {args.precision}, plans {plan_s:.1f}s",
          file=sys.stderr, flush=True)

    def step():
        out, _, _ = ctx.sample_batch(pts, n, plans=plans, precision=prec, capacity=cap)
        return out, ctx.timing()

    for w in range(args.warmup):
        _, tm = step()
        print(f"warmup {w}: {tm['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc, decide_ms, out, tm = 0, [], None, None
    t0 = time.perf_counter()
    for s in range(args.steps):
        out, tm = step()
        acc += sum(int(o["n_accepted"]) for o in out)
        decide_ms.append(tm["decide_ms"] / max(tm["decide_launches"], 1))
        print(f"step {s}: {tm['total_ms']:.1f} ms, decide {tm['decide_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_prop = n_per * len(pts) * args.steps
    avg_decide_s = sum(decide_ms) / len(decide_ms) / 1e3
    per_launch = n_per * len(pts)
    ops = method_ops_per_proposal(K, "sigma", args.precision)
    roof = alu_roof(ops * per_launch / avg_decide_s, traffic=load_traffic(K, args.precision, per_launch,
                                                                           "k_decide128"),
                    kernel=f"k_decide128<{K}>", method_ops_per_proposal=ops, avg_launch_ms=avg_decide_s * 1e3,
                    proposals_per_launch=per_launch,
                    **mfma_fields(K, args.precision, "sigma", per_launch / avg_decide_s))
    n_cpu = ((1 << 16) if K == 64 else (1 << 15)) if args.cpu_sample < 0 else args.cpu_sample
    cpu = None
    if n_cpu > 0:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(specs, plans, n_cpu)
    line = {
        "metric": f"accepted samples/sec at K={K} (plain Sigma proposal); proposals/sec",
        "value": acc / dt, "unit": "accepted samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_label(args.precision), "data": "synthetic",
        "config": {"workload": workload, "K": K, "N": 4 * K, "points": len(pts), "proposals_per_point": n_per,
                   "synthesis": args.precision, "fp64_redecision": True},
        "proposals_per_s": n_prop / dt, "acceptance": acc / n_prop,
        "per_point": [{"beta_p": s.beta_p, "level": s.beta_p * s.c32, "acceptance": int(o["n_accepted"]) / n_per,
                       "skewness": o["skewness"], "kurtosis": o["kurtosis"],
                       "fp64_redecisions": int(o["n_fp64_fixups"])} for s, o in zip(specs, out)],
        "plan_seconds": plan_s,
        "phase_ms_last_step": {k: round(v, 3) for k, v in tm.items() if k.endswith("_ms")},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def learned_bench(args) -> int:
    import math

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        return 1
    from scipy import stats as sst

    from paper_2411_16952_amd import learned
    from paper_2411_16952_amd import tkdv as T
    from paper_2411_16952_amd import workloads as W

    prec = T.PRECISIONS[args.precision]
    ctx = T.Context(0)
    train = [T.make_point(s.K, s.E0, s.beta_p, s.c32, seed=s.seed, point_id=s.point_id)
             for s in W.learned_train_points()]
    K = train[0].K
    seeds = [int(v) for v in args.train_seeds.split(",")]
    cfgs = [T.learner_cfg(K, hidden=256, eps=W.LEARNED_EPS, v_amp=0.5, v_scale=1.0, lr=3e-3, seed=sd) for sd in seeds]
    t0 = time.perf_counter()
    ens = learned.fit_ensemble(ctx, train, cfgs, samples_per_point=4096, rounds=args.train_rounds,
                               steps=args.train_steps, max_proposals=1 << 36, precision=prec,
                               log=lambda m: print("train " + m, file=sys.stderr, flush=True))
    train_s = time.perf_counter() - t0
    train_gains = [math.exp(float(np.mean(r.history[r.best_round]["log_gain"]))) for r in ens]

    specs = W.learned_eval_points()
    pts = [T.make_point(s.K, s.E0, s.beta_p, s.c32, seed=s.seed, point_id=s.point_id) for s in specs]
    t0 = time.perf_counter()
    # M_mix of every network at every point (searched on the GPU); each point samples with the
    # network whose M_mix there is smallest
    mixes, mplans, splans, chosen = learned.plan_for_points_ensemble(ctx, ens, pts, margin=0.02)
    plan_s = time.perf_counter() - t0
    log_gain = [learned.log_M_sigma_normalised(sp) - pl.log_M for sp, pl in zip(splans, mplans)]
    n_per = int(args.proposals)
    cap = 1 << 20
    print(f"bench: learned vs plain, {len(pts)} points, K={K}, {n_per:.3g} proposals/point/sampler, "
          f"{args.precision}; training {train_s:.1f}s, plans {plan_s:.1f}s; M_Sigma/M_mix geometric mean "
          f"{math.exp(sum(log_gain) / len(log_gain)):.1f}", file=sys.stderr, flush=True)

    def mix_step():
        out, dec_ms, launches = [], 0.0, 0
        for p, pl, mx in zip(pts, mplans, mixes):
            out.append(ctx.sample_mixture(p, pl, mx, n_per, precision=prec, capacity=cap))
            tm = ctx.timing()
            dec_ms += tm["decide_ms"]
            launches += tm["decide_launches"]
        return out, dec_ms, launches

    def plain_step():
        out, _, _ = ctx.sample_batch(pts, [n_per] * len(pts), plans=splans, precision=prec,
                                     capacity=[cap] * len(pts))
        return out, ctx.timing()

    for w in range(args.warmup):
        mix_step()
        plain_step()
        print(f"warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc_m, dec_ms_m, launches_m, out_m = 0, 0.0, 0, None
    t0 = time.perf_counter()
    for s in range(args.steps):
        out_m, dms, nl = mix_step()
        acc_m += sum(int(o["n_accepted"]) for o in out_m)
        dec_ms_m += dms
        launches_m += nl
        print(f"mixture step {s}: {acc_m} accepted so far", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt_m = time.perf_counter() - t0
    acc_p, out_p = 0, None
    t0 = time.perf_counter()
    for s in range(args.steps):
        out_p, tm = plain_step()
        acc_p += sum(int(o["n_accepted"]) for o in out_p)
        print(f"plain step {s}: {tm['total_ms']:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    n_prop = n_per * len(pts) * args.steps

    # exactness at equal accuracy: u(0) of the two samplers' stored samples, per level
    ks = {}
    for lvl in W.LEARNED_EVAL_LEVELS:
        idx = [i for i, s in enumerate(specs) if abs(s.beta_p * s.c32 - lvl) < 1e-6 * lvl]
        pv = []
        for i in idx:
            xm = out_m[i]["xhat"][:20000].double().cpu().numpy()
            xp = out_p[i]["xhat"][:20000].double().cpu().numpy()
            if len(xm) > 20 and len(xp) > 20:
                pv.append(float(sst.ks_2samp(xm[:, :K].sum(1), xp[:, :K].sum(1)).pvalue))
        ks[f"{lvl:g}"] = {"min_p": min(pv) if pv else None, "median_p": float(np.median(pv)) if pv else None,
                          "points": len(pv)}

    # roofline of the dominant kernel: k_decide_mix, one launch per point
    avg_launch_s = dec_ms_m / max(launches_m, 1) / 1e3
    ops = method_ops_per_proposal(K, "mixture", args.precision)
    achieved = ops * n_per / avg_launch_s
    roof = alu_roof(achieved, traffic=load_traffic(K, args.precision, n_per, "k_decide_mix"),
                    kernel="k_decide_mix", method_ops_per_proposal=ops,
                    avg_launch_ms=avg_launch_s * 1e3, proposals_per_launch=n_per,
                    **mfma_fields(K, args.precision, "mixture", n_per / avg_launch_s))

    n_cpu = (1 << 17) if args.cpu_sample < 0 else args.cpu_sample
    cpu = cpu_plain = None
    if n_cpu > 0:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline_mixture(specs, mixes, mplans, n_cpu)
        cpu_plain = cpu_baseline(specs, splans, n_cpu)

    per_point = [{"beta_p": s.beta_p, "level": s.beta_p * s.c32, "M_gain": math.exp(g),
                  "acc_mixture": int(om["n_accepted"]) / n_per, "acc_plain": int(op["n_accepted"]) / n_per,
                  "fp64_redecisions": int(om["n_fp64_fixups"]), "M_violations": int(om["n_M_violations"])}
                 for s, g, om, op in zip(specs, log_gain, out_m, out_p)]
    line = {
        "metric": "accepted samples/sec at K=32 (learned-mixture vs plain proposal); proposals/sec",
        "value": acc_m / dt_m,
        "unit": "accepted samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_m / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_label(args.precision),
        "data": "synthetic",
        "config": {
            "workload": "learned mixture vs plain Sigma: K=32, N=128, E0=1, 16 beta' in [20, 60] x "
                        "beta'C3/C2 in {9000, 12000} (32 points), 1e9 proposals/point per sampler; networks "
                        "3-256-256-160 fitted on beta'C3/C2 = 9000 (other seeds), eps = 0.2; per point the "
                        "network with the smallest rejection constant",
            "K": K, "N": 4 * K, "points": len(pts), "proposals_per_point": n_per,
            "synthesis": args.precision, "fp64_redecision": True,
        },
        "training": {"seconds": train_s, "network_seeds": seeds, "train_points_M_gain": train_gains,
                     "networks_chosen": [seeds[c] for c in chosen],
                     "selection": "per evaluation point, the network with the smallest M_mix (plan time)"},
        "plain_value": acc_p / dt_p,
        "ratio_vs_plain": (acc_m / dt_m) / (acc_p / dt_p) if acc_p else None,
        "proposals_per_s": n_prop / dt_m,
        "plain_proposals_per_s": n_prop / dt_p,
        "acceptance": acc_m / n_prop,
        "plain_acceptance": acc_p / n_prop,
        "M_gain_geomean": math.exp(sum(log_gain) / len(log_gain)),
        "M_violations_last_step": sum(int(o["n_M_violations"]) for o in out_m),
        "ks_u0_mixture_vs_plain": ks,
        "train_seconds": train_s,
        "plan_seconds": plan_s,
        "per_point": per_point,
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_plain": cpu_plain,
    }
    print(json.dumps(line), flush=True)
    for r in ens:
        r.learner.close()
    ctx.close()
    return 0


def sweep_bench(args) -> int:
    """The batched sweep: 256 points of mixed K with accepted targets, windows
    replayed as a hipGraph, launch configuration from the autotuner."""
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X GPU", file=sys.stderr)
        return 1
    from paper_2411_16952_amd import tkdv as T
    from paper_2411_16952_amd import workloads as W

    prec = T.PRECISIONS[args.precision]
    ctx = T.Context(0)
    t0 = time.perf_counter()
    tuned = {K: ctx.autotune(K, prec, args.tune_cache).to_dict() for K in (16, 32, 64)}
    tune_s = time.perf_counter() - t0
    print(f"autotune {tune_s:.1f}s: {tuned}", file=sys.stderr, flush=True)
    # screen the seeded candidates: acceptance >= 1e-4 on 1e6 proposals
    t0 = time.perf_counter()
    kept, kept_plans = [], []
    cands = W.sweep_candidates()
    plan_s = 0.0

    def alpha_root_exists(p):  # a root of F exists iff beta' < K^2 sum_k 1/k^2 (Sec. III.A)
        return p.beta_p < p.K * p.K * sum(1.0 / (k * k) for k in range(1, p.K + 1))

    for b0 in range(0, len(cands), 64):
        batch = [sp for sp in cands[b0:b0 + 64] if alpha_root_exists(sp.point)]
        cpts = [T.make_point(sp.point.K, sp.point.E0, sp.point.beta_p, sp.point.c32, seed=sp.point.seed,
                             point_id=sp.point.point_id) for sp in batch]
        tp = time.perf_counter()
        cplans, _ = ctx.plan_batch(cpts, T.SIGMA, n_starts=16, seed=2024)   # log M searched on the GPU
        plan_s += time.perf_counter() - tp
        out, _, _ = ctx.sample_batch(cpts, [10**6] * len(cpts), plans=cplans, precision=prec)
        for sp, p, pl, o in zip(batch, cpts, cplans, out):
            if o["n_accepted"] >= 100 and len(kept) < W.SWEEP_N:
                kept.append((sp, p))
                kept_plans.append(pl)
        if len(kept) >= W.SWEEP_N:
            break
    screen_s = time.perf_counter() - t0
    pts = [p for _, p in kept]
    targets = [int(sp.target) for sp, _ in kept]
    maxp = [W.SWEEP_CAP] * len(pts)
    caps = [min(t, 1 << 14) for t in targets]
    Ks = [p.K for p in pts]
    print(f"sweep: {len(pts)} points (K=16: {Ks.count(16)}, 32: {Ks.count(32)}, 64: {Ks.count(64)}), "
          f"targets sum {sum(targets):.3g}; screening {screen_s:.1f}s", file=sys.stderr, flush=True)

    def step():
        return ctx.sample_sweep(pts, targets, maxp, plans=kept_plans, precision=prec, capacity=caps)[0]

    for w in range(args.warmup):
        step()
        print(f"warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    acc = prop = 0
    ops = 0.0
    windows, graph_launches = [], []
    t0 = time.perf_counter()
    for s in range(args.steps):
        out = step()
        windows.append(ctx.timing()["windows"])
        graph_launches.append(ctx.timing()["graph_launches"])
        acc += sum(int(o["n_accepted"]) for o in out)
        prop += sum(int(o["n_proposed"]) for o in out)
        ops += sum(method_ops_per_proposal(p.K, "sigma", args.precision) * int(o["n_proposed"])
                   for p, o in zip(pts, out))
        print(f"sweep step {s}: {ctx.timing()['total_ms']:.0f} ms, {windows[-1]} windows", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    met = sum(int(o["n_accepted"]) >= t for o, t in zip(out, targets))
    roof = alu_roof(ops / dt, traffic=None, kernel="k_decide (all K, whole sweep)",
                    note="method-level ops of all proposals over the whole sweep's wall time (every phase), a "
                         "lower bound on the decide kernels' own rate")
    n_cpu = (1 << 12) if args.cpu_sample < 0 else args.cpu_sample
    cpu = cpu_baseline(pts, kept_plans, n_cpu) if n_cpu > 0 else None
    line = {
        "metric": "accepted samples/sec, batched sweep (256 points, K in {16,32,64}, accepted targets)",
        "value": acc / dt, "unit": "accepted samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_label(args.precision), "data": "synthetic",
        "config": {"workload": "batched sweep: 256 points, K uniform in {16,32,64}, beta' ~ U[10,80], E0 in "
                               "{0.5,1,pi/2,2}, beta'C3/C2 sqrt(E0) ~ U[0, P_max(K)], acceptance >= 1e-4, "
                               "targets log-uniform in [1e4,1e6], cap 1e10 proposals/point, windows as hipGraph "
                               "replays", "points": len(pts), "targets_sum": sum(targets),
                   "synthesis": args.precision},
        "proposals_per_s": prop / dt, "targets_met": met, "windows_per_step": windows,
        "graph_launches_per_step": graph_launches,
        "autotuned": {str(k): v for k, v in tuned.items()}, "autotune_seconds": tune_s,
        "screen_seconds": screen_s, "plan_seconds": plan_s, "plan": "GPU multi-start search (tkdv_plan_batch, 16 starts)",
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="learned", choices=["learned", "plain", "sweep", "sir", "k64", "k128"])
    ap.add_argument("--tune-cache", default="/tmp/tkdv_autotune.txt", help="autotuner cache (sweep workload)")
    ap.add_argument("--proposals", type=float, default=1e9, help="proposals per point (per sampler)")
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3"],
                    help="synthesis products of the sampling workloads (plain BF16 takes no decisions)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="oracle proposals per point (0: skip; default 2^22 plain, 2^17 learned)")
    ap.add_argument("--train-rounds", type=int, default=6)
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--train-seeds", default=",".join(str(v) for v in range(1, 25)),
                    help="network initialisations trained; each evaluation point samples with the network "
                         "whose rejection constant there is smallest")
    ap.add_argument("--synthesis", action="store_true",
                    help="only time the standalone synthesis kernel (K = 64, N = 256, 2^20 rows of x^ "
                         "in HBM) for FP32, BF16 and BF16x3 products; prints one JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy, "copies": 3}))
        return 0
    if args.synthesis:
        return synthesis_bench(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sampler's proposals "
              "are independent, and multi-GPU sharding is a design note, not a measured path.",
              file=sys.stderr)
        return 2

    if args.workload == "sweep":
        return sweep_bench(args)
    if args.workload == "sir":
        return sir_bench(args)
    if args.workload in QUARTER_WORKLOADS:
        return quarter_bench(args)
    return learned_bench(args) if args.workload == "learned" else plain_bench(args)


if __name__ == "__main__":
    sys.exit(main())
