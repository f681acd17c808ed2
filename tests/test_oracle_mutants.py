"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/julia_oracle.c, changes one line the way a plausible
slip would (a dropped term, a wrong sign, an off-by-one index, a non-strict
comparison, a lost error term), builds the copy on the CPU into a temporary
directory and runs a fast subset of the pins of test_oracle_pins.py against
it.  Every mutant has to fail at least one pin; the real oracle passes them all.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins
from oracle import build_oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "julia_oracle.c")

MUTANTS = {
    "non_strict_escape": ("if (m > 4.0)\n            break;\n        double re",
                          "if (m >= 4.0)\n            break;\n        double re"),
    "general_non_strict": ("if (m > 4.0)\n            break;\n        double wr",
                           "if (m >= 4.0)\n            break;\n        double wr"),
    "minus_cr": ("double xn = re + cr;", "double xn = re - cr;"),
    "plus_y2": ("double re = x2 - y2;", "double re = x2 + y2;"),
    "dropped_two": ("double tx = 2.0 * x;", "double tx = x;"),
    "ci_to_cr": ("double yn = im + ci;", "double yn = im + cr;"),
    "row_flip": ("*y = cy - py;", "*y = cy + py;"),
    "pixel_corner": ("double oi = (double)(2 * (int64_t)i + 1 - W);",
                     "double oi = (double)(2 * (int64_t)i - W);"),
    "hx_off_by_one": ("double hx = (re_max - re_min) / (2.0 * (double)W);",
                      "double hx = (re_max - re_min) / (2.0 * (double)W - 2.0);"),
    "cap_plus_one": ("    while (n < max_iter) {\n        double x2 = x * x;\n        double y2 = y * y;\n"
                     "        double m = x2 + y2;\n        if (m > 4.0)\n            break;\n"
                     "        double re",
                     "    while (n <= max_iter) {\n        double x2 = x * x;\n        double y2 = y * y;\n"
                     "        double m = x2 + y2;\n        if (m > 4.0)\n            break;\n"
                     "        double re"),
    "fp32_unfused_norm": ("float m = fmaf(y, y, t);", "float m = y * y + t;"),
    "fp32_unshifted_limit": ("const float lim = 4.0f + cr;", "const float lim = 4.0f;"),
    "fp32_sign": ("float xn = fmaf(-y, y, t);", "float xn = fmaf(y, y, t);"),
    "ff_lost_sl": ("float c = sl + th;", "float c = th;"),
    "ff_lost_cross": ("float cross = fmaf(x.lo, y.hi, cross1);", "float cross = cross1;"),
    "ff_lost_tl": ("float w = tl + vl;", "float w = vl;"),
    "ff_escape_lo": ("(m.hi == 4.0f && m.lo <= 0.0f)", "(m.hi == 4.0f)"),
    "ff_sqr_lost_cross": ("float q = fmaf(twice_hi, x.lo, e);", "float q = e;"),
    "ff_sqr_once": ("float twice_hi = x.hi + x.hi;", "float twice_hi = x.hi;"),
    "ff_sqr_lost_err": ("float q = fmaf(twice_hi, x.lo, e);", "float q = twice_hi * x.lo;"),
    "ff_cheap_lost_lows": ("float err = sl + lows;", "float err = sl;"),
    "ff_cheap_lost_sl": ("float err = sl + lows;", "float err = lows;"),
    "ff_cheap_lost_ylo": ("float lows = x.lo + y.lo;", "float lows = x.lo;"),
    "colour_level_shift": ("out[k] = palette[level];",
                           "out[k] = palette[level > 0 ? level - 1 : 0];"),
    "colour_clamp_to_first": ("            level = palette_len - 1;", "            level = 0;"),
    "general_sign": ("double nr = p_rr - p_ii;", "double nr = p_rr + p_ii;"),
    "general_cross": ("double ni = p_ri + p_ir;", "double ni = p_ri - p_ir;"),
    "general_degree": ("for (int32_t k = 1; k < d; k++) {\n            double p_rr",
                       "for (int32_t k = 2; k < d; k++) {\n            double p_rr"),
    "general_fp32_sign": ("float nr = p_rr - p_ii;", "float nr = p_rr + p_ii;"),
    "general_ff_cross": ("dw p_ir = dw_mul(wi, x);", "dw p_ir = dw_mul(wi, y);"),
    "mandel_z0_is_c": ("return jro_count(dtype, 0.0, 0.0, x, y, max_iter);",
                       "return jro_count(dtype, x, y, x, y, max_iter);"),
    # the per-pixel entry points: column and row swapped, width and height
    # swapped, the list index shifted by one, the mode dropped
    "pixels_ij_swap": ("                             W, H, max_iter, ii[k], jj[k]);",
                       "                             W, H, max_iter, jj[k], ii[k]);"),
    "pixels_general_ij_swap": ("im_max, W, H, max_iter, ii[k], jj[k]);",
                               "im_max, W, H, max_iter, jj[k], ii[k]);"),
    "pixels_general_wh_swap": ("im_max, W, H, max_iter, ii[k], jj[k]);",
                               "im_max, H, W, max_iter, ii[k], jj[k]);"),
    "pixels_index_shift": ("                             W, H, max_iter, ii[k], jj[k]);",
                           "                             W, H, max_iter, ii[k], jj[k > 0 ? k - 1 : 0]);"),
    "pixels_mode_dropped": ("        out[k] = pixel_count(dtype, mode, cr, ci,",
                            "        out[k] = pixel_count(dtype, JRO_JULIA, cr, ci,"),
    # the two-parameter rational maps: a pole's 0/0 taken as bounded, a sign
    # in lam conj(W), |W|^2 with a minus, Im(lam / W) dropped, lam's parts
    # swapped (FP32), the per-pixel entry's column and row swapped
    "rational_nan_inside": ("if (!(m <= 4.0))", "if (m > 4.0)"),
    "rational_re_sign": ("double num_r = a + b;", "double num_r = a - b;"),
    "rational_im_sign": ("double num_i = e - f;", "double num_i = f - e;"),
    "rational_norm_sign": ("double q = q_r + q_i;", "double q = q_r - q_i;"),
    "rational_dropped_im": ("double si = wi + ci;\n        x = sr + tr;\n        y = si + ti;",
                            "double si = wi + ci;\n        x = sr + tr;\n        y = si;"),
    "rational_fp32_lambda_parts": ("float a = lr * wr;", "float a = li * wr;"),
    "rational_pixels_ij_swap": ("W, H, ii[k], jj[k], &x, &y);", "W, H, jj[k], ii[k], &x, &y);"),
    # the prescribed cardioid path: 2u lost, a growing instead of shrinking,
    # the conjugate step, the bits of k taken lowest first, u^2 with a sign
    "cardioid_no_two": ("double nr = 2.0 * pr - wr;", "double nr = pr - wr;"),
    "cardioid_a_plus": ("double a = a0 - dk;", "double a = a0 + dk;"),
    "cardioid_conj_step": ("cmul(pr, pi, step_re, step_im, &pr, &pi);",
                           "cmul(pr, pi, step_re, -step_im, &pr, &pi);"),
    "cardioid_bit_order": ("for (int32_t bit = 30; bit >= 0; bit--) {\n        cmul(pr",
                           "for (int32_t bit = 0; bit <= 30; bit++) {\n        cmul(pr"),
    "cardioid_square_sign": ("    *re = ac - bd;\n    *im = ad + bc;", "    *re = ac + bd;\n    *im = ad + bc;"),
}


def _battery():
    """Fast subset of the pins; returns the names of those that fail."""
    failed = []
    checks = [("orbits_" + d, pins.test_exact_small_orbits, (d,)) for d in pins.DTYPES]
    checks += [("numpy_%s_%d" % (d, k), pins.test_matches_numpy_reimplementation, (d, k))
               for d in pins.DTYPES for k in (1, 3)]
    checks += [("fingerprint", pins.test_c1_fingerprint, ()),
               ("centres", pins.test_pixel_centres, ()),
               ("sub_ulp_escape", pins.test_escape_by_less_than_fp32_ulp, ()),
               ("fp32_formulation", pins.test_fp32_escape_test_formulation, ()),
               ("cap01_fp64", pins.test_cap_zero_and_one, ("fp64",)),
               ("eft", pins.test_error_free_transforms, ()),
               ("colour_table", pins.test_colorize_literal_table, ()),
               ("general_orbits_fp64", pins.test_general_exact_small_orbits, ("fp64",)),
               ("general_orbits_fp32", pins.test_general_exact_small_orbits, ("fp32",)),
               ("general_orbits_ff", pins.test_general_exact_small_orbits, ("ff",)),
               ("general_quadratic", pins.test_general_degree_two_is_the_quadratic_map_fp64, ()),
               ("general_numpy_fp32_3", pins.test_general_matches_numpy_reimplementation,
                ("fp32", 3)),
               ("general_numpy_ff_3", pins.test_general_matches_numpy_reimplementation,
                ("ff", 3)),
               ("dw_bounds", pins.test_double_word_error_bounds, ()),
               ("dw_cheap_bounds", pins.test_cheap_double_word_error_bounds, ())]
    checks += [("pixels_%s_%d_%d" % (d, case, deg), pins.test_render_pixels_matches_whole_images,
                (d, case, deg))
               for d, case, deg in (("fp64", 0, 2), ("fp32", 1, 2), ("ff", 0, 3), ("fp64", 1, 5))]
    checks += [("rational_orbits_" + d, pins.test_rational_exact_small_orbits, (d,))
               for d in pins.RATIONAL_DTYPES]
    checks += [("rational_numpy_%s_%d" % (d, k), pins.test_rational_matches_numpy_reimplementation,
                (d, k)) for d, k in (("fp64", 2), ("fp32", 3))]
    checks += [("rational_pixels_fp64", pins.test_render_pixels_rational_matches_whole_images,
                ("fp64",))]
    checks += [("cardioid_exact", pins.test_cardioid_constants_exact_quarter_turns, ()),
               ("cardioid_mp", pins.test_cardioid_constants_against_high_precision, ())]
    for name, fn, args in checks:
        try:
            fn(*args)
        except AssertionError:
            failed.append(name)
    return failed


@pytest.fixture
def swap_lib():
    saved = oracle._load()
    yield
    oracle._lib = saved


def test_real_oracle_passes_battery():
    assert _battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, swap_lib):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, "mutation site must be unique: %r" % old
    src = tmp_path / "julia_oracle.c"
    src.write_text(text.replace(old, new))
    (tmp_path / "julia_oracle.h").write_text(open(SRC[:-2] + ".h").read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *build_oracle.CFLAGS, str(src), "-o", str(lib), "-lm"],
                   check=True, capture_output=True)
    oracle._lib = oracle._open(str(lib))
    failed = _battery()
    assert failed, "mutant %s passed every pin" % name
