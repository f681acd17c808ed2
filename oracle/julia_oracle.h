/*
 * julia_oracle.h -- plain CPU oracle for escape-time Julia / Mandelbrot counts.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the definition of the method.  It shares no code, header, table or
 * helper with the GPU library; only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  Nothing in the product path calls it.
 *
 * Method (Mayfield et al., "Fractal Art Generation using GPUs", Section 2):
 * every pixel of the image is scaled onto a window of the complex plane to give
 * an initial point Z_0; the map Z_{n+1} = Z_n^2 + C is iterated and the pixel
 * records how many iterations it takes to diverge, with a cap on the number of
 * iterations (the paper's cap is 100).  Section 3: in the Mandelbrot variant
 * the pixel supplies C and Z_0 = 0.
 *
 * Readings of the paper taken here (the paper leaves them open):
 *   - count = index n of the first iterate with |Z_n|^2 > 4 (strict), tested
 *     as fl(fl(x*x) + fl(y*y)) > 4 before Z_n is advanced; count = max_iter if
 *     no iterate below max_iter escapes; max_iter = 0 gives 0 everywhere.
 *   - pixel (i, j) (column i, row j, row 0 on top) has its centre at
 *       x = cx + (2i + 1 - W) * hx,   y = cy - (2j + 1 - H) * hy
 *     with hx = (re_max - re_min) / (2W), hy = (im_max - im_min) / (2H),
 *     cx = (re_min + re_max) / 2, cy = (im_min + im_max) / 2; every product is
 *     rounded before the sum (no fused multiply-add).
 *   - the FP64 update is x' = (x*x - y*y) + cr, y' = ((2x) * y) + ci, each
 *     operation rounded to binary64.
 *   - FP32 and float-float are two further arithmetic formulations of the same
 *     iteration, fixed here so that a GPU kernel using them can be checked
 *     bit for bit (see julia_oracle.c).  Float-float squares with the
 *     double-word square, multiplies 2x by y with the double-word product,
 *     and sums with the cheaper double-word sum (jro_dw_sqr, jro_dw_mul,
 *     jro_dw_add_cheap); the general maps' float-float uses the accurate
 *     double-word sum and product (jro_dw_add, jro_dw_mul) throughout.
 *
 * All functions are synchronous, single-threaded and take host pointers.
 * Arguments are not validated: callers pass W, H >= 1 and max_iter >= 0.
 */
#ifndef JULIA_ORACLE_H
#define JULIA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic formulations. */
#define JRO_FP64 0
#define JRO_FP32 1
#define JRO_FF   2

/* Which quantity the pixel supplies. */
#define JRO_JULIA      0 /* Z_0 = pixel, C = given constant      (Section 2) */
#define JRO_MANDELBROT 1 /* Z_0 = 0,     C = pixel               (Section 3) */

/* Full image, row-major (H rows of W counts), row 0 = im_max. */
void jro_render(int32_t dtype, int32_t mode, double cr, double ci,
                double re_min, double re_max, double im_min, double im_max,
                int32_t W, int32_t H, int32_t max_iter, int32_t *out);

/* Counts of n listed pixels (column ii[k], row jj[k]) of the same image. */
void jro_render_pixels(int32_t dtype, int32_t mode, double cr, double ci,
                       double re_min, double re_max, double im_min, double im_max,
                       int32_t W, int32_t H, int32_t max_iter, int64_t n,
                       const int32_t *ii, const int32_t *jj, int32_t *out);

/* Centre of pixel (i, j) in binary64. */
void jro_pixel_center(double re_min, double re_max, double im_min, double im_max,
                      int32_t W, int32_t H, int32_t i, int32_t j,
                      double *x, double *y);

/* Count for one orbit with explicit Z_0 = x0 + i y0 and C = cr + i ci
 * (both given in binary64 and converted per formulation). */
int32_t jro_count(int32_t dtype, double x0, double y0, double cr, double ci,
                  int32_t max_iter);

/* General maps (the paper's further functions, Section 4 and its closing
 * future work): Z_{n+1} = Z_n^d + C for an integer degree d in 2..8, the
 * same count, escape test and pixel mapping.  Z^d is formed by d - 1 complex
 * products W <- W * Z from W = Z, each product (a + ib)(x + iy) taken as
 * (a*x - b*y) + i (a*y + b*x) with every operation rounded; then C is added.
 * FP64 and FP32 use that order in their own precision (no fused operations;
 * the test is fl(fl(x*x) + fl(y*y)) > 4); float-float uses the double-word
 * product and sum for every operation.  For d = 2 the FP64 result equals
 * jro_count's except where x*y is subnormal. */
int32_t jro_count_general(int32_t dtype, int32_t degree, double x0, double y0,
                          double cr, double ci, int32_t max_iter);
void jro_render_general(int32_t dtype, int32_t mode, int32_t degree, double cr, double ci,
                        double re_min, double re_max, double im_min, double im_max,
                        int32_t W, int32_t H, int32_t max_iter, int32_t *out);
void jro_render_pixels_general(int32_t dtype, int32_t mode, int32_t degree, double cr,
                               double ci, double re_min, double re_max, double im_min,
                               double im_max, int32_t W, int32_t H, int32_t max_iter,
                               int64_t n, const int32_t *ii, const int32_t *jj, int32_t *out);

/* Rational maps with two complex parameters (the further functions and
 * parameters of Section 4 and the closing discussion):
 *     Z_{n+1} = W + C + lambda / W,   W = Z_n^d,  d = 2..8,
 * Julia images only (the pixel gives Z_0), FP64 or FP32.  W is formed as in
 * the general maps; lambda / W as (Re(lambda conj W) + i Im(lambda conj W)) /
 * |W|^2 with
 *     |W|^2 = wr*wr + wi*wi,  Re = lr*wr + li*wi,  Im = li*wr - lr*wi,
 * each product, sum and quotient rounded in the formulation's precision (no
 * fused operations; IEEE division); then
 *     x' = (wr + cr) + Re/|W|^2,   y' = (wi + ci) + Im/|W|^2.
 * Count and pixel mapping as above; the test is "escaped unless
 * fl(fl(x*x) + fl(y*y)) <= 4", so an iterate that is not a number (Z = 0 is
 * a pole: 0/0) counts as escaped.  With lambda = 0 the counts are those of
 * Z^d + C wherever no iterate is exactly 0. */
int32_t jro_count_rational(int32_t dtype, int32_t degree, double x0, double y0, double cr,
                           double ci, double lr, double li, int32_t max_iter);
void jro_render_rational(int32_t dtype, int32_t degree, double cr, double ci, double lr,
                         double li, double re_min, double re_max, double im_min,
                         double im_max, int32_t W, int32_t H, int32_t max_iter, int32_t *out);
void jro_render_pixels_rational(int32_t dtype, int32_t degree, double cr, double ci,
                                double lr, double li, double re_min, double re_max,
                                double im_min, double im_max, int32_t W, int32_t H,
                                int32_t max_iter, int64_t n, const int32_t *ii,
                                const int32_t *jj, int32_t *out);

/* Prescribed parameter path (Section 3): the constant of frame k on the
 * cardioid f(t) = ((2 cos t - cos 2t) / a, (2 sin t - sin 2t) / a), which is
 * (2u - u^2) / a for u = e^{it}, with a changing along the path:
 *     u_k = step^k by square-and-multiply over the bits of k, highest first
 *           (p = 1; for each bit: p = p*p, then p = p*step if the bit is set),
 *     a_k = a0 - da * k,
 *     C_k = (2 u_k - u_k*u_k) / a_k,
 * every complex product (a + ib)(c + id) taken as (a*c - b*d) + i (a*d + b*c),
 * and every product, sum and quotient rounded to binary64.  step = e^{i dt}
 * is given (the caller forms it once); a decreasing a grows the cardioid. */
void jro_cardioid_constant(double step_re, double step_im, double a0, double da, int32_t k,
                           double *cr, double *ci);

/* Colour levels from counts (Section 2: each pixel is given a colour level by
 * its iteration count): out[k] = palette[min(counts[k], palette_len - 1)],
 * for counts >= 0 and palette_len >= 1. */
void jro_colorize(const int32_t *counts, int64_t n, const uint32_t *palette,
                  int32_t palette_len, uint32_t *out);

/* Float-float building blocks, exported so that their error-free and
 * error-bound properties can be checked against exact rational arithmetic. */
void jro_two_sum(float a, float b, float *s, float *e);
void jro_fast_two_sum(float a, float b, float *s, float *e);
void jro_two_prod(float a, float b, float *p, float *e);
void jro_dw_add(float xh, float xl, float yh, float yl, float *zh, float *zl);
void jro_dw_mul(float xh, float xl, float yh, float yl, float *zh, float *zl);
void jro_dw_split(double v, float *hi, float *lo);
/* The cheaper square and sum of the quadratic map's float-float iteration
 * (julia_oracle.c): TwoProd of the high part plus one fused 2*hi*lo term;
 * TwoSum of the high parts plus the low parts, one Fast2Sum. */
void jro_dw_sqr(float xh, float xl, float *zh, float *zl);
void jro_dw_add_cheap(float xh, float xl, float yh, float yl, float *zh, float *zl);

#ifdef __cplusplus
}
#endif

#endif /* JULIA_ORACLE_H */
