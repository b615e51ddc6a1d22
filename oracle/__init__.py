"""CPU FP64 oracle for the TKdV Gibbs rejection sampler (arXiv 2411.16952).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it, and
this package never imports the product package: the two share no code.

Layout:
  * ``tkdv_oracle.c`` -- per-proposal arithmetic in plain C, IEEE double
    precision, one proposal at a time (Philox4x32-10 words, Box-Muller normals,
    projection onto the sphere, H2 by Parseval, H3 by the paper's double sum,
    the acceptance ratio, the accept loop, ensemble statistics).
  * ``core.py`` -- ctypes bindings of that library.
  * ``plan.py`` -- the per-point precompute of the algorithm's step 1: the root
    alpha* of F, the proposal variances and the rejection constant M.

Parity status of each function is recorded in the module docstrings; every
function here is pinned by the ``-m "not gpu"`` tests under ``tests/``.
"""
from .core import (  # noqa: F401
    OracleStats,
    lib,
    philox4x32_10,
    proposal_words,
    uniform_of_word,
    normals,
    t_of,
    H2,
    H3_triad,
    H3_quad,
    grid,
    log_ratio,
    F_alpha,
    proposal,
    sample,
    sample_until,
    eval_batch,
    MIX_S,
    MIX_R,
    make_mixture,
    shift,
    mix_log_q,
    mix_draw,
    mix_sample,
    mix_proposal,
    extremes,
    sir,
    mix_eps,
    mix_threshold,
    stats_of,
    hist_bin,
    max_threads,
)
from .plan import OraclePlan, alpha_star, sigma2, log_M, plan_point  # noqa: F401
