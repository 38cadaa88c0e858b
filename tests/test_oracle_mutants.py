"""Planted mistakes: each mutant is a copy of the oracle with one plausible bug
(built on the CPU only).  Every mutant must fail at least one pin of
``test_oracle_pins`` -- evidence that the pins constrain each part of the oracle.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

import pytest

from oracle import oracle
from tests import test_oracle_pins as pins

MUTANTS = {
    "philox_key_bump": ("k1 += W1;", "k1 += W0;"),
    "philox_word_order": ("uint32_t n1 = (uint32_t)p1;", "uint32_t n1 = (uint32_t)p0;"),
    "u24_fifth_slot": ("((w[1] & 0xFFu) << 8)", "((w[1] & 0xFFu) << 9)"),
    "uniform_offset": ("((double)u + 0.5) * 0x1p-24", "((double)u) * 0x1p-24"),
    "no_row_swap": ("if (p11 * p22 - p12 * p21 < 0.0) {", "if (0) {"),
    "swap_not_undone": ("if (swapped) {", "if (0 && swapped) {"),
    "scaling_transposed": ("double s11 = p11 / p12;", "double s11 = p11 / p21;"),
    "remark_sign": ("double sphi = a / (sqrt(1.0 + a) + sqrt(1.0 - a));",
                    "double sphi = a / (sqrt(1.0 + a) - sqrt(1.0 - a));"),
    "remark_cos": ("double cphi = 0.5 * (sqrt(1.0 + a) + sqrt(1.0 - a));",
                   "double cphi = 0.5 * (sqrt(1.0 + a) + sqrt(1.0 - a * a));"),
    "theorem_alpha_from_C": ("par[0] = log(B21 / B11);", "par[0] = log(C21 / C11);"),
    "theorem_beta_sign": ("par[3] = log((B22 * B11) / (B12 * B21));",
                          "par[3] = -log((B22 * B11) / (B12 * B21));"),
    "odds_ratio_sign": ("L[a * q_max + b] + L[0] - L[a * q_max + 0] - L[b]",
                        "L[a * q_max + b] - L[0] - L[a * q_max + 0] - L[b]"),
    "rrow_transposed": ("rr[a] = L[a * q_max + 0] - L[0];", "rr[a] = L[0 * q_max + a] - L[0];"),
    "dual_bits_swapped": ("int y = (x_src == a), yp = (x_dst == b);",
                          "int y = (x_dst == b), yp = (x_src == a);"),
    "dual_threshold_direction": ("return !(u < p0);", "return u < p0;"),
    "dual_index_stride": ("int d = (a - 1) * (qj - 1) + (b - 1);\n            if (d % 5 == 0)",
                          "int d = (a - 1) * (qi - 1) + (b - 1);\n            if (d % 5 == 0)"),
    "primal_side1_uses_beta1": ("s += pe[d * 5 + 1] + thd * pe[d * 5 + 4];",
                                "s += pe[d * 5 + 1] + thd * pe[d * 5 + 3];"),
    "primal_side0_index": ("int d = (a - 1) * (qo - 1) + (b - 1);\n                    int thd",
                           "int d = (b - 1) * (qo - 1) + (a - 1);\n                    int thd"),
    "cdf_not_normalised": ("if (u * F[qn - 1] < F[a]) { x = a; break; }",
                           "if (u < F[a]) { x = a; break; }"),
    "cdf_not_cumulative": ("F[a] = acc;", "F[a] = exp(L[a] - mx);"),
    "primal_node_quad_word": ("(int)(node % 4));", "(int)(c % 4));"),
    "logv_sign": ("out[c] = log_p - log_cond;", "out[c] = log_p + log_cond;"),
    "logv_no_shift": ("log_cond += L[x[i * C + c]] - (mx + log(z));",
                      "log_cond += L[x[i * C + c]] - log(z);"),
    "logv_edge_transposed": ("log_p += Lam[(e * q_max + a) * q_max + b];",
                             "log_p += Lam[(e * q_max + b) * q_max + a];"),
    "dual_flag_on_p_theta1": ("*flag = fabs(u - p0) < ORC_FLAG_BAND;",
                              "*flag = fabs(u - (1.0 - p0)) < ORC_FLAG_BAND;"),
    "flag_band_wide": ("#define ORC_FLAG_BAND 1e-6", "#define ORC_FLAG_BAND 1e-4"),
    "cdf_flag_unnormalised": ("if (fabs(u - F[k] / F[qn - 1]) < ORC_FLAG_BAND) f = 1;",
                              "if (fabs(u - F[k]) < ORC_FLAG_BAND) f = 1;"),
    "cdf_flag_includes_one": ("for (int k = 0; k + 1 < qn; ++k)\n        if (fabs(u",
                              "for (int k = 0; k < qn; ++k)\n        if (fabs(u"),
    "init_floor": ("x[i * C + c] = (uint8_t)floor(u * q[i]);",
                   "x[i * C + c] = (uint8_t)floor(u * (q[i] - 1));"),
}

FAST_PINS = [
    pins.test_philox_known_answers,
    pins.test_uniform_mapping_and_balance,
    pins.test_factor2x2_reconstructs_every_positive_table,
    pins.test_factor2x2_symmetric_case_is_the_lemma_in_trig_form,
    pins.test_theorem_params_mixture_equals_table,
    lambda: [pins.test_ising_closed_form(J) for J in (-0.3, 0.3)],
    lambda: [pins.test_decomposition_mixture_reconstructs_table(a, b) for a, b in ((4, 3), (3, 4))],
    lambda: [pins.test_exact_transition_detailed_balance_and_stationarity(n, m)
             for n, m in pins._tiny_models()],
    lambda: [pins.test_sampler_matches_exact_transition_rows(a, b) for a, b in ((3, 4), (4, 2))],
    lambda: [pins.test_dual_draw_frequencies_match_conditional(a, b) for a, b in ((3, 4), (4, 2))],
    lambda: [pins.test_dual_flag_band_sits_on_p_theta0(J) for J in (0.3, 1.1)],
    lambda: [pins.test_categorical_flag_band_sits_on_normalised_cdf(w, s)
             for w, s in (([1.0, 2.0, 3.0, 4.0], 5.0), ([1.0, 3.0], -2.0))],
    lambda: pins.test_flag_rate_is_the_band_width("ising"),
    pins.test_equal_weights_draw_is_floor_uq,
    pins.test_init_is_floor_uq,
    lambda: [pins.test_log_v_estimator_identities_by_enumeration(n, m)
             for n, m in pins._tiny_models()],
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    find, repl = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(find) == 1, f"mutation site not unique for {name}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        open(path, "w").write(src.replace(find, repl))
        subprocess.check_call(["gcc", *oracle.FLAGS, "-o", so, path, "-lm"])
        oracle.use_library(so)
        try:
            caught = []
            for pin in FAST_PINS:
                try:
                    pin()
                except (AssertionError, ValueError, FloatingPointError):
                    caught.append(getattr(pin, "__name__", "pin"))
            assert caught, f"mutant {name} passed every pin"
        finally:
            oracle.use_library(None)
