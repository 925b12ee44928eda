"""Planted mistakes: copies of the oracle compiled with one plausible error
each (reversed sort, dropped term, transposed slot index, short chunk
maximum, truncating rounding, a wrong |A||x| scale, ...) must each fail at
least one pin. The mistakes live only in temporary copies; the oracle itself
is untouched."""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_oracle_crs as crs_pins
import test_oracle_rounding as rnd_pins
import test_oracle_sell as sell_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "sort_ascending": ("if (p->len != q->len) return p->len > q->len ? -1 : 1;",
                       "if (p->len != q->len) return p->len > q->len ? 1 : -1;",
                       [lambda: sell_pins.test_global_sort_is_stable_length_sort_and_maximises_beta(),
                        lambda: sell_pins.test_worst_case_beta(4, 64)]),
    "ties_reversed": ("return (p->row > q->row) - (p->row < q->row);",
                      "return (p->row < q->row) - (p->row > q->row);",
                      [lambda: sell_pins.test_global_sort_is_stable_length_sort_and_maximises_beta()]),
    "dropped_last_term": ("for (int64_t j = rpt[i]; j < rpt[i + 1]; ++j) s += val[j] * x[col[j]];\n      y[i] = s;\n    }\n  } else {",
                          "for (int64_t j = rpt[i]; j + 1 < rpt[i + 1]; ++j) s += val[j] * x[col[j]];\n      y[i] = s;\n    }\n  } else {",
                          [lambda: crs_pins.test_laplacian_row_sums(128),
                           lambda: crs_pins.test_threads_do_not_change_bits(),
                           lambda: crs_pins.test_powerlaw_within_bound_of_companion()]),
    "sign_error": ("s += (long double)val[j] * (long double)x[col[j]];",
                   "s -= (long double)val[j] * (long double)x[col[j]];",
                   [lambda: crs_pins.test_integer_matrix_equals_dense_matvec((33, 40), False)]),
    "transposed_slot": ("int64_t idx = cs[i] + j * C + r;\n        int64_t p = i * C + r;",
                        "int64_t idx = cs[i] + r * cl[i] + j;\n        int64_t p = i * C + r;",
                        [lambda: sell_pins.test_sell_spmv_equals_crs_spmv_bitwise(32, 1),
                         lambda: sell_pins.test_invariants_random(4, 3, 1)]),
    "short_chunk_max": ("for (int64_t r = 0; r < C; ++r) {\n      int64_t p = i * C + r;\n      if (p < n) {",
                        "for (int64_t r = 0; r + 1 < C; ++r) {\n      int64_t p = i * C + r;\n      if (p < n) {",
                        [lambda: sell_pins.test_stencil27_beta_closed_form(24, 8),
                         lambda: sell_pins.test_staircase_beta(8)]),
    "window_off_by_one": ("for (int64_t w0 = 0; w0 < n; w0 += sigma) {\n    int64_t w1 = w0 + sigma < n ? w0 + sigma : n;",
                          "for (int64_t w0 = 0; w0 < n; w0 += sigma + 1) {\n    int64_t w1 = w0 + sigma + 1 < n ? w0 + sigma + 1 : n;",
                          [lambda: sell_pins.test_invariants_random(8, 16, 2)]),
    "bf16_truncates": ("r = ldexp(rint(q), qexp);", "r = ldexp(trunc(q), qexp);",
                       [lambda: rnd_pins.test_bf16_golden_cases()]),
    "bf16_spacing_off": ("int qexp = (e - 1) - 7;", "int qexp = (e - 1) - 8;",
                         [lambda: rnd_pins.test_bf16_golden_cases()]),
    "symperm_forward_map": ("col2[k] = iperm[col[j]];", "col2[k] = perm[col[j]];",
                            [lambda: sell_pins.test_symmetric_permutation_identity(4),
                             lambda: sell_pins.test_symmetric_permutation_identity(100)]),
    "block_form_wrong_stride": ("(long double)X[(int64_t)col[j] * k + v];", "(long double)X[(int64_t)col[j] + v];",
                                [lambda: crs_pins.test_block_form_columns_match_single_vector()]),
    "absmv_no_fabs_x": ("s += fabsl((long double)val[j]) * fabsl((long double)x[col[j]]);",
                        "s += fabsl((long double)val[j]) * ((long double)x[col[j]]);",
                        [lambda: crs_pins.test_absmv_exact_rational(2, 26, 26),
                         lambda: crs_pins.test_absmv_two_sided_bound(5)]),
    "absmv_doubled": ("s += fabsl((long double)val[j]) * fabsl((long double)x[col[j]]);",
                      "s += 2 * fabsl((long double)val[j]) * fabsl((long double)x[col[j]]);",
                      [lambda: crs_pins.test_absmv_exact_rational(1, 10, 10),
                       lambda: crs_pins.test_absmv_two_sided_bound(6)]),
    "absmv_first_column": ("s += fabsl((long double)val[j]) * fabsl((long double)x[col[j]]);",
                           "s += fabsl((long double)val[j]) * fabsl((long double)x[col[rpt[i]]]);",
                           [lambda: crs_pins.test_absmv_exact_rational(3, 30, 28),
                            lambda: crs_pins.test_absmv_two_sided_bound(5)]),
    "f32_truncates": ("for (int64_t t = 0; t < count; ++t) out[t] = (float)in[t];",
                      "for (int64_t t = 0; t < count; ++t) {\n    float f_ = (float)in[t];\n"
                      "    if (fabs((double)f_) > fabs(in[t])) f_ = nextafterf(f_, 0.0f);\n    out[t] = f_;\n  }",
                      [lambda: rnd_pins.test_f32_golden_cases()]),
    "f32_flushes_subnormals": ("for (int64_t t = 0; t < count; ++t) out[t] = (float)in[t];",
                               "for (int64_t t = 0; t < count; ++t)\n"
                               "    out[t] = fabs(in[t]) < 0x1p-126 ? copysignf(0.0f, (float)in[t]) : (float)in[t];",
                               [lambda: rnd_pins.test_f32_golden_cases()]),
    "zeta_wrong_mean": ("long double d = (long double)(rpt[i + 1] - rpt[i]) - mean;",
                        "long double d = (long double)(rpt[i + 1] - rpt[i]) - mean + 1;",
                        [lambda: sell_pins.test_zeta_closed_form()]),
}


@pytest.fixture
def mutant_lib(tmp_path):
    built = []

    def make(name):
        old, new, _ = MUTANTS[name]
        src = open(SRC).read()
        assert src.count(old) == 1, "mutation site for %s not unique" % name
        path = tmp_path / ("oracle_%s.c" % name)
        path.write_text(src.replace(old, new))
        so = tmp_path / ("liboracle_%s.so" % name)
        subprocess.check_call(["gcc", *oracle.CFLAGS, str(path), "-o", str(so), "-lm"])
        lib = oracle.configure(ctypes.CDLL(str(so)))
        built.append(lib)
        return lib

    saved = oracle._lib
    yield make
    oracle._lib = saved


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, mutant_lib):
    lib = mutant_lib(name)
    oracle._lib = lib
    caught = 0
    for pin in MUTANTS[name][2]:
        try:
            pin()
        except AssertionError:
            caught += 1
    assert caught > 0, "no pin failed for the planted mistake %s" % name
