"""Planted mistakes in a copy of the oracle must each fail a pin.

Each case edits one line of a temporary copy of ``oracle/tkdv_oracle.c`` (a
sign, an index, a dropped factor, a swapped function), builds it, and runs the
fast subset of ``test_oracle_pins.py`` against that build in a subprocess.  The
pins pass on the real oracle (that is ``test_oracle_pins.py`` itself); here
every mutant must make at least one of them fail (the mixture and SIR
mutants run against their own pin files).  Mistakes in the Philox constants,
word order and round count are caught by the generator's published
known-answer vectors.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tkdv_oracle.c")

FAST_PINS = " or ".join([
    "appendix_A", "dirichlet_kernel", "double_sum_equals", "parseval", "H3_odd",
    "box_muller", "philox_known", "uniform_sphere_law", "K2_brute_force", "uniform_proposal_linear",
    "paper_linear_rows and 16-", "positive_nonlinearity", "extremes_",
])

MUTATIONS = {
    "triad_product_sign": ("in_re += p_re * q_re - p_im * q_im;", "in_re += p_re * q_re + p_im * q_im;"),
    "triad_index": ("double q_re = a * xh[n - k - 1], q_im = -a * xh[K + n - k - 1];",
                    "double q_re = a * xh[n - k - 1], q_im = -a * xh[K + n - k];"),
    "triad_no_conjugate": ("total += n_re * in_re + n_im * in_im;", "total += n_re * in_re - n_im * in_im;"),
    "triad_prefactor": ("return 2.0 * M_PI * total;", "return M_PI * total;"),
    "t_dropped_square": ("t += (double)k * k * s;", "t += (double)k * s;"),
    "g_sign": ("lr += K * log1p(alpha * beta_p * orc_t(K, xh) / K3);",
               "lr -= K * log1p(alpha * beta_p * orc_t(K, xh) / K3);"),
    "sigma_power": ("return 1.0 / (1.0 + alpha * beta_p * (double)k * k / K3);",
                    "return 1.0 / (1.0 + alpha * beta_p * (double)k / K3);"),
    "sigma_index": ("scale = sqrt(orc_sigma2(K, p->beta_p, p->alpha_star, m % K + 1));",
                    "scale = sqrt(orc_sigma2(K, p->beta_p, p->alpha_star, m / 2 + 1));"),
    "grid_sin_as_cos": ("s += xh[k - 1] * cos(k * xi) + xh[K + k - 1] * sin(k * xi);",
                        "s += xh[k - 1] * cos(k * xi) + xh[K + k - 1] * cos(k * xi);"),
    "philox_multipliers_swapped": (
        "uint64_t prod_a = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;\n        uint64_t prod_b = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;",
        "uint64_t prod_a = (uint64_t)PHILOX_MUL_B * (uint64_t)x0;\n        uint64_t prod_b = (uint64_t)PHILOX_MUL_A * (uint64_t)x2;"),
    "philox_weyl_constant": ("static const uint32_t PHILOX_WEYL_B = 0xBB67AE85u;",
                             "static const uint32_t PHILOX_WEYL_B = 0xBB67AE87u;"),
    "philox_word_order": ("uint32_t y0 = hi_b ^ x1 ^ k0;", "uint32_t y0 = hi_a ^ x1 ^ k0;"),
    "philox_nine_rounds": ("for (int round = 0; round < 10; ++round) {", "for (int round = 0; round < 9; ++round) {"),
    "box_muller_pair": ("z[2 * m + 1] = r * sin(th);", "z[2 * m + 1] = r * cos(th);"),
    "box_muller_radius": ("double r = sqrt(-2.0 * log(u1));", "double r = sqrt(-log(u1));"),
    "hamiltonian_sign": ("return beta_p / (E0 * (double)K * K) * (H2 - c32 * H3);",
                         "return beta_p / (E0 * (double)K * K) * (H2 + c32 * H3);"),
    "hamiltonian_scale": ("return beta_p / (E0 * (double)K * K) * (H2 - c32 * H3);",
                          "return beta_p / (E0 * (double)K) * (H2 - c32 * H3);"),
    "stats_cube": ("st->S3 += u2 * u;", "st->S3 += u2 * u2;"),
    "hist_bins": ("double pos = (u0 + u_max) / (2.0 * u_max) * ORC_NBINS;",
                  "double pos = (u0 + u_max) / (2.0 * u_max) * (ORC_NBINS - 1);"),
    "accept_rule": ("acc[q] = (uint8_t)(lu < la);", "acc[q] = (uint8_t)(lu < la + 0.05);"),
    "four_sigma_scale": ("g->four_sigma = 4.0 * sqrt(E0 / M_PI);", "g->four_sigma = 4.0 * sqrt(E0 / (2 * M_PI));"),
    "max4_counts_values": ("if (umax > g->four_sigma) st->n_max4++;", "if (umax > g->two_sigma) st->n_max4++;"),
    "peak_keeps_last_tie": ("if (umax > st->peak_u) {", "if (umax >= st->peak_u) {"),
    "peak_index_offset": ("stats_add_sample(&local, &g, xh, i0 + q);", "stats_add_sample(&local, &g, xh, q);"),
}


# mistakes in the learned-proposal functions, run against the mixture pins
MIX_PINS = " or ".join(["normalised", "dense_definition", "V0_and_D_sigma", "shift_group",
                        "draw_has_density", "component_weights"])
MIX_MUTATIONS = {
    "mix_woodbury_sign": ("double e = w[c] - (m->V[c][0] * g[0] + m->V[c][1] * g[1]);",
                          "double e = w[c] + (m->V[c][0] * g[0] + m->V[c][1] * g[1]);"),
    "mix_logdet_half": ("return -0.5 * logdet_L0 - K * log(qf);", "return -logdet_L0 - K * log(qf);"),
    "mix_gram_identity": ("double G[ORC_MIX_R][ORC_MIX_R] = {{1.0, 0.0}, {0.0, 1.0}};",
                          "double G[ORC_MIX_R][ORC_MIX_R] = {{1.0, 0.0}, {0.0, 0.0}};"),
    "mix_weights_swapped": ("double a = log(eps) + lg, b = log1p(-eps) + lnet;",
                            "double a = log1p(-eps) + lg, b = log(eps) + lnet;"),
    "mix_draw_sqrt_d": ("X[c] = exp(0.5 * m->logd[c % K]) * z[c] + rv0[c] * eta[0] + rv1[c] * eta[1];",
                        "X[c] = exp(m->logd[c % K]) * z[c] + rv0[c] * eta[0] + rv1[c] * eta[1];"),
    "mix_draw_eta": ("X[c] = exp(0.5 * m->logd[c % K]) * z[c] + rv0[c] * eta[0] + rv1[c] * eta[1];",
                     "X[c] = exp(0.5 * m->logd[c % K]) * z[c] + rv0[c] * eta[0] + rv1[c] * eta[0];"),
    "mix_shift_pair": ("out[K + k - 1] = b * c - a * s;", "out[K + k - 1] = b * c + a * s;"),
    "mix_component_rule": ("comp = (int)((wc - E) / B);", "comp = (int)((wc - E) / B / 2);"),
}


# mistakes in the sampling-importance resampling, run against its pins
SIR_PINS = " or ".join(["equal_weights", "parseval_moments", "rejection_probabilities", "systematic_resampling",
                        "agrees_with_rejection"])
SIR_MUTATIONS = {
    "sir_weight_power": ("        w[q] = exp(la);\n", "        w[q] = exp(2.0 * la);\n"),
    "sir_no_offset": ("double pos = (u0 + (double)r) * W / (double)m;", "double pos = (double)r * W / (double)m;"),
    "sir_unweighted_moments": ("for (int c = 0; c < 4; ++c) M[c] += w[q] * mom[4 * q + c];",
                               "for (int c = 0; c < 4; ++c) M[c] += mom[4 * q + c];"),
    "sir_fourth_power": ("s4 += u * u * u * u;", "s4 += u * u * u;"),
    "sir_second_sum": ("W2 += w[q] * w[q];", "W2 += w[q];"),
}


def _run_mutant(name, old, new, pins_file, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        c_path = os.path.join(d, "mut.c")
        so_path = os.path.join(d, "libmut.so")
        with open(c_path, "w") as f:
            f.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", so_path,
                        c_path, "-lm"], check=True)
        env = dict(os.environ, TKDV_ORACLE_LIB=so_path, OMP_NUM_THREADS="4")
        return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                               os.path.join(ROOT, "tests", pins_file), "-k", pins],
                              cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name", sorted(MIX_MUTATIONS))
def test_planted_mixture_mistake_is_caught(name):
    old, new = MIX_MUTATIONS[name]
    r = _run_mutant(name, old, new, "test_mixture_oracle.py", MIX_PINS)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(SIR_MUTATIONS))
def test_planted_sir_mistake_is_caught(name):
    old, new = SIR_MUTATIONS[name]
    r = _run_mutant(name, old, new, "test_sir_oracle.py", SIR_PINS)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        c_path = os.path.join(d, "mut.c")
        so_path = os.path.join(d, "libmut.so")
        with open(c_path, "w") as f:
            f.write(src.replace(old, new))
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", so_path,
                        c_path, "-lm"], check=True)
        env = dict(os.environ, TKDV_ORACLE_LIB=so_path, OMP_NUM_THREADS="4")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", FAST_PINS],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
