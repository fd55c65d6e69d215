"""The pins catch plausible slips in the oracle.

Each case plants one mistake (in the arithmetic or in the |term| sums
that the parity gates divide by) in a private copy of the oracle's C source (on
the CPU, in a temporary directory), builds it, swaps it in for the real
oracle, and checks that at least one pin of test_oracle_pins.py fails.  The
real oracle is restored afterwards.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "rsm_oracle.c")

MUTATIONS = {
    "truncated_mod": ("    if (q < 0) q += m;\n", ""),
    "dropped_origin": ("int64_t v = t->origin[d];", "int64_t v = 0;"),
    "transposed_paving": ("t->paving[d * rep_rank + k] * r[k]",
                          "t->paving[k * t->arr_rank + d] * r[k]"),
    "dropped_fitting": ("v += t->fitting[d * t->pat_rank + k] * i[k];", "(void)i;"),
    "transposed_fitting": ("t->fitting[d * t->pat_rank + k] * i[k]",
                           "t->fitting[k * t->arr_rank + d] * i[k]"),
    "column_major_linearisation": ("lin = lin * t->shape[d] + floor_mod(v, t->shape[d]);",
                                   "lin += floor_mod(v, t->shape[d]) * "
                                   "(d ? t->shape[d - 1] : 1);"),
    "reversed_weights": ("if (kind == OR_WSUM) term *= coeffs[pf];",
                         "if (kind == OR_WSUM) term *= coeffs[np - 1 - pf];"),
    "dot_same_operand": ("* x[1][element_offset(&in[1], rep_rank, r, i2)];",
                         "* x[0][element_offset(&in[0], rep_rank, r, i)];"),
    "adjoint_sign": ("gx[a] += c * g;", "gx[a] -= c * g;"),
    "adjoint_weight_grad_uses_weight": ("gc[jf * np + pf] += g * x[a];", "gc[jf * np + pf] += c * x[a];"),
    "adjoint_drops_weight": ("gx[a] += c * g;", "gx[a] += g;"),
    "csr_first_column_only": ("double term = vals[k] * x[col_idx[k]];",
                              "double term = vals[k] * x[col_idx[row_ptr[r]]];"),
    "cg_initial_residual_sign": ("r[i] = b[i] - q[i];", "r[i] = b[i] + q[i];"),
    "cg_residual_update_sign": ("r[i] -= alpha * q[i];", "r[i] += alpha * q[i];"),
    "cg_beta_inverted": ("const double beta = rho_next / rho;",
                         "const double beta = rho / rho_next;"),
    "cg_direction_from_residual": ("p[i] = r[i] + beta * p[i];", "p[i] = r[i] + beta * r[i];"),
    "cg_absolute_stop": ("sqrt(rho) > tol * bnorm", "sqrt(rho) > tol"),
    # slips in the |term| sums that every FP32 parity gate divides by
    "wsum_bound_drops_weight": ("            if (kind == OR_WSUM) term *= coeffs[pf];\n"
                                "            acc += term;\n"
                                "            aabs += fabs(term);",
                                "            aabs += fabs(term);\n"
                                "            if (kind == OR_WSUM) term *= coeffs[pf];\n"
                                "            acc += term;"),
    "dot_bound_abs_of_sum": ("* x[1][element_offset(&in[1], rep_rank, r, i2)];\n"
                             "            acc += term;\n"
                             "            aabs += fabs(term);",
                             "* x[1][element_offset(&in[1], rep_rank, r, i2)];\n"
                             "            acc += term;\n"
                             "            aabs = fabs(acc);"),
    "adjoint_gx_bound_scaled": ("gx_abs[a] += fabs(c * g);", "gx_abs[a] += 10.0 * fabs(c * g);"),
    "adjoint_gc_bound_scaled": ("gc_abs[jf * np + pf] += fabs(g * x[a]);",
                                "gc_abs[jf * np + pf] += 10.0 * fabs(g * x[a]);"),
    "copy_bound_signed": ("yabs[pf] = fabs(y[pf]);", "yabs[pf] = y[pf];"),
    # slips in the weighted sum with an output pattern of several elements
    "multi_output_transposed_taps": ("double term = coeffs[jf * np + pf] * x[0]",
                                     "double term = coeffs[pf * n_out + jf] * x[0]"),
    "multi_output_first_row_only": ("double term = coeffs[jf * np + pf] * x[0]",
                                    "double term = coeffs[pf] * x[0]"),
    "multi_output_bound_drops_weight": ("                acc += term;\n                aabs += fabs(term);\n"
                                        "            }\n            y[jf] = acc;",
                                        "                acc += term;\n                aabs += fabs(term / coeffs[jf * np + pf]);\n"
                                        "            }\n            y[jf] = acc;"),
    "multi_output_adjoint_transposed_taps": ("double c = coeffs ? coeffs[jf * np + pf] : 1.0;",
                                             "double c = coeffs ? coeffs[pf * nq + jf] : 1.0;"),
    "multi_output_adjoint_first_phase_gradient": ("double g = gy[element_offset(out_t, rep_rank, r, j)];",
                                                  "j[0] = 0; double g = gy[element_offset(out_t, rep_rank, r, j)];"),
}

PINS = [
    pins.test_indices_hand_example_negative_origin,
    pins.test_indices_hand_example_2d_transposed_roles,
    pins.test_indices_match_numpy_wrap_ravel_random_tilers,
    pins.test_small_sum_equals_block_reshape_sum,
    pins.test_two_stage_equals_einsum,
    pins.test_matmul_tilers_equal_naive_triple_loop,
    pins.test_adjoint_identity_random_tilers,
    pins.test_finite_differences_match_chain_adjoint,
    pins.test_csr_matches_scipy_and_dense,
    pins.test_cg_solution_matches_dense_solve,
    pins.test_cg_iterates_match_scipy,
    pins.test_cg_stopping_rule_is_relative,
    pins.test_wsum_and_sum_abs_sums_match_index_table_random_tilers,
    pins.test_dot_abs_sum_equals_naive_loop_on_absolutes,
    pins.test_dot_abs_sum_random_tiler_pairs,
    pins.test_copy_abs_sum_is_magnitude,
    pins.test_adjoint_abs_sums_match_index_table_random_tilers,
    pins.test_adjoint_abs_sums_two_stage_closed_form,
    pins.test_polyphase_forward_equals_fft_correlation_per_phase,
    pins.test_polyphase_one_hot_taps_select_samples,
    pins.test_polyphase_adjoint_equals_fft_and_adjoint_identity,
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, "mutation anchor vanished: " + name
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", str(so),
                           str(mutant_src), "-lm"])
    real = oracle._load()
    oracle._lib = oracle._bind(ctypes.CDLL(str(so)))
    caught = []
    try:
        for pin in PINS:
            try:
                pin()
            except (AssertionError, ValueError):
                caught.append(pin.__name__)
                break
    finally:
        oracle._lib = real
    assert caught, "no pin caught mutation " + name
