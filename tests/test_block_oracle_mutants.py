"""Planted mistakes in the learned-block-proposal oracle: each mutant is a copy
of ``oracle/block_oracle.py`` with one plausible bug; every mutant must fail at
least one pin of ``test_block_oracle_pins``."""
from __future__ import annotations

import os
import types

import pytest

from oracle import block_oracle
from tests import test_block_oracle_pins as pins

SRC = block_oracle.__file__

MUTANTS = {
    "cut_field_beta_of_other_end": ("f_node[i] += dec.rrow[e, 1] + a1 + th * b1",
                                    "f_node[i] += dec.rrow[e, 1] + a1 + th * b2"),
    "cut_field_without_rescaling": ("f_node[j] += dec.rcol[e, 1] + a2 + th * b2",
                                    "f_node[j] += a2 + th * b2"),
    "internal_shift_transposed": ("f_node[i] += Lam[e, 1, 0] - Lam[e, 0, 0]",
                                  "f_node[i] += Lam[e, 0, 1] - Lam[e, 0, 0]"),
    "coupling_sign": ("Lam[e, 1, 1] + Lam[e, 0, 0] - Lam[e, 1, 0] - Lam[e, 0, 1]",
                      "Lam[e, 1, 1] - Lam[e, 0, 0] - Lam[e, 1, 0] - Lam[e, 0, 1]"),
    "cut_dual_direction": ("theta[e] = (~(u[k] < p0))", "theta[e] = ((u[k] < p0))"),
    "cut_dual_endpoints_swapped": ("y = x[model.src[e]].astype", "y = x[model.dst[e]].astype"),
    "accept_proposal_ratio_sign": ("((np.asarray(xb, float) - np.asarray(xpb, float)) * logits)",
                                   "((np.asarray(xpb, float) - np.asarray(xb, float)) * logits)"),
    "accept_target_ratio_missing": ("return log_ptilde(xpb, f, K) - log_ptilde(xb, f, K)",
                                    "return log_ptilde(xb, f, K) - log_ptilde(xb, f, K)"),
    "proposal_direction": ("xp = (u[..., :k] < p1)", "xp = (u[..., :k] > p1)"),
    "relu_mask_dropped": ('dH2 = r((dL @ P["W3"]) * (H2 > 0))', 'dH2 = r((dL @ P["W3"]))'),
    "grad_w1_transposed_input": ('g["W1"], g["b1"] = dH1.T @ X, dH1.sum(0)',
                                 'g["W1"], g["b1"] = dH1.T @ X * 0.5, dH1.sum(0)'),
    "adam_no_bias_correction": ("mh = m / (1 - beta1 ** step)", "mh = m"),
    "bf16_truncates": ("u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16", "u = u >> 16 << 16"),
}

PINS = [
    pins.test_block_conditional_is_the_mrf_given_cut_duals,
    lambda: [pins.test_mh_kernel_detailed_balance_and_stationarity(2, 5)],
    pins.test_exact_proposal_is_always_accepted,
    pins.test_sampled_transitions_match_the_mh_matrix,
    pins.test_learned_step_leaves_the_joint_invariant,
    pins.test_mlp_gradients_match_finite_differences,
    pins.test_adam_first_step_closed_form,
    pins.test_bf16_rounding_is_nearest_even,
    pins.test_cut_dual_frequencies_match_the_dual_conditional,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_block_mutant_is_caught(name):
    find, repl = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(find) == 1, f"mutation site not unique for {name}"
    mod = types.ModuleType("oracle.block_oracle_mutant")
    mod.__package__ = "oracle"
    mod.__file__ = os.path.join(os.path.dirname(SRC), "block_oracle_mutant.py")
    exec(compile(src.replace(find, repl), mod.__file__, "exec"), mod.__dict__)
    saved = pins.B
    pins.B = mod
    try:
        caught = []
        for pin in PINS:
            try:
                pin()
            except (AssertionError, ValueError, FloatingPointError, IndexError):
                caught.append(getattr(pin, "__name__", "pin"))
        assert caught, f"mutant {name} passed every pin"
    finally:
        pins.B = saved
