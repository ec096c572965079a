"""Plausible mistakes planted in copies of the oracle (on the CPU) must each be
caught by at least one pin.  This shows the pins constrain every part of the
definition: sign and index of each term, transposition, conjugation (with and
without transposition), the strides, the scalar policies (including the
literal interpretation of a complex alpha) and the real-C projection."""
import os
import shutil

import pytest

import oracle
import oracle_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "md_oracle.c")

MUTANTS = {
    "re_sign": ("sr += ar * br - ai * bi;", "sr += ar * br + ai * bi;"),
    "im_sign": ("si += ar * bi + ai * br;", "si += ar * bi - ai * br;"),
    "im_term_dropped": ("si += ar * bi + ai * br;", "si += ar * bi;"),
    "no_conj": ("*im = -*im;", "(void)0;"),
    "trans_ignored": ("fetch(X, dt, rs, cs, p, i, re, im);", "fetch(X, dt, rs, cs, i, p, re, im);"),
    "index_transposed": ("int64_t idx = r * rs + c * cs;", "int64_t idx = r * cs + c * rs;"),
    "row_stride_ignored": ("int64_t idx = r * rs + c * cs;", "int64_t idx = r + c * cs;"),
    "r_op_not_conjugated": ("if (tr == 'C' || tr == 'R')", "if (tr == 'C')"),
    "r_op_transposed": ("if (tr == 'N' || tr == 'R')", "if (tr == 'N')"),
    "alpha_cross_sign": ("double tr = use_ab ? alpha_re * sr - alpha_im * si : 0.0;",
                         "double tr = use_ab ? alpha_re * sr + alpha_im * si : 0.0;"),
    "beta_imag_kept_for_real_c": ("double bim = tag_complex(dtc) ? beta_im : 0.0;",
                                  "double bim = beta_im;"),
    "real_c_keeps_imag": ("*out_im = tag_complex(dtc) ? ri : 0.0;", "*out_im = ri;"),
    "alpha_rule_case0": ("return alpha_im != 0.0 && cs != 0 && cs != 7;",
                         "return alpha_im != 0.0 && cs != 7;"),
    "beta_conj": ("rr = bre * cr - bim * ci + tr;", "rr = bre * cr + bim * ci + tr;"),
    "c_read_when_beta_zero": ("if (bre != 0.0 || bim != 0.0) {", "if (1) {"),
    "single_promoted_wrong": ("*im = (double)((const float *)X)[2 * idx + 1];",
                              "*im = (double)((const float *)X)[2 * idx];"),
    "last_k_dropped": ("for (int64_t p = 0; p < k; ++p) {", "for (int64_t p = 0; p + 1 < k; ++p) {"),
    "literal_still_refuses": ("if (!literal && alpha_refused(dtc, dta, dtb, alpha_im))",
                              "if (alpha_refused(dtc, dta, dtb, alpha_im))"),
    "alpha_projected_in_mixed_cases": ("if (md_oracle_case(dtc, dta, dtb) == 0)",
                                       "if (md_oracle_case(dtc, dta, dtb) != 7)"),
    "half_exponent_bias": ("v = ldexp((double)(1024 + f), e - 25);", "v = ldexp((double)(1024 + f), e - 24);"),
    "half_implicit_bit_dropped": ("v = ldexp((double)(1024 + f), e - 25);", "v = ldexp((double)f, e - 15);"),
    "half_subnormal_scale": ("v = ldexp((double)f, -24);", "v = ldexp((double)f, -25);"),
    "half_complex_parts_swapped": ("*im = half_value(((const uint16_t *)X)[2 * idx + 1]);",
                                   "*im = half_value(((const uint16_t *)X)[2 * idx]);"),
    "bound_term_doubled": ("g += sqrt(ar * ar + ai * ai) * sqrt(br * br + bi * bi);",
                           "g += 2.0 * sqrt(ar * ar + ai * ai) * sqrt(br * br + bi * bi);"),
    "bound_term_l1": ("g += sqrt(ar * ar + ai * ai) * sqrt(br * br + bi * bi);",
                      "g += (fabs(ar) + fabs(ai)) * (fabs(br) + fabs(bi));"),
    "bound_term_real_parts": ("g += sqrt(ar * ar + ai * ai) * sqrt(br * br + bi * bi);",
                              "g += fabs(ar) * fabs(br);"),
    "gemm_at_rows_cols_swapped": ("beta_re, beta_im, C, dtc, 1, ldc, rows[t], cols[t],",
                                  "beta_re, beta_im, C, dtc, 1, ldc, cols[t], rows[t],"),
    "flops_case2": ("double f = (ncomplex <= 1) ? 2.0 : (ncomplex == 2 ? 4.0 : 8.0);",
                    "double f = (ncomplex <= 1) ? 2.0 : (ncomplex == 2 ? 8.0 : 8.0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + old
    shutil.copy(os.path.join(os.path.dirname(SRC), "md_oracle.h"), tmp_path / "md_oracle.h")
    (tmp_path / "mut.c").write_text(src.replace(old, new))
    lib = oracle.build(str(tmp_path / "mut.c"), str(tmp_path / "libmut.so"))
    res = oracle_pins.run_all(oracle.Oracle(lib))
    caught = [k for k, v in res.items() if v]
    assert caught, "mutant %s passed every pin" % name
