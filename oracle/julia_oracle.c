/*
 * julia_oracle.c -- plain, slow, single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see julia_oracle.h): used by tests, the smoke
 * check and the benchmark's CPU-baseline leg; never by the product path.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (oracle/build_oracle.py).  -ffp-contract=off keeps every a*b + c of the
 * FP64 and FP32 paths as a rounded product followed by a rounded sum; fused
 * multiply-adds appear only where fmaf() is called by name.  On x86-64 the
 * float and double types evaluate in their own precision (SSE), so every
 * operation below is one IEEE-754 round-to-nearest-even operation.
 *
 * Source of the method: Mayfield et al., Section 2 (escape-time iteration of
 * Z_{n+1} = Z_n^2 + C over pixels scaled onto the complex plane, iteration
 * cap) and Section 3 (Mandelbrot variant: C from the pixel, Z_0 = 0).
 */
#include "julia_oracle.h"

#include <math.h>

/* ------------------------------------------------------------------------ */
/* Pixel -> complex plane ("region-covering routine", Section 2).            */
/* The pixel centre is cx + (2i+1-W)*hx; row 0 is the top of the window.     */
/* ------------------------------------------------------------------------ */
void jro_pixel_center(double re_min, double re_max, double im_min, double im_max,
                      int32_t W, int32_t H, int32_t i, int32_t j,
                      double *x, double *y)
{
    double hx = (re_max - re_min) / (2.0 * (double)W);
    double hy = (im_max - im_min) / (2.0 * (double)H);
    double cx = 0.5 * (re_min + re_max);
    double cy = 0.5 * (im_min + im_max);
    double oi = (double)(2 * (int64_t)i + 1 - W);
    double oj = (double)(2 * (int64_t)j + 1 - H);
    double px = oi * hx;
    double py = oj * hy;
    *x = cx + px;
    *y = cy - py;
}

/* ------------------------------------------------------------------------ */
/* FP64: the definition itself.                                              */
/* n counts how many times Z has been advanced; the loop stops at the first  */
/* iterate with |Z|^2 > 4 or when n reaches the cap.                         */
/* ------------------------------------------------------------------------ */
static int32_t count_fp64(double x, double y, double cr, double ci, int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        double x2 = x * x;
        double y2 = y * y;
        double m = x2 + y2;
        if (m > 4.0)
            break;
        double re = x2 - y2;
        double xn = re + cr;        /* Re(Z^2 + C) */
        double tx = 2.0 * x;        /* exact */
        double im = tx * y;
        double yn = im + ci;        /* Im(Z^2 + C) = 2xy + Im C */
        x = xn;
        y = yn;
        n = n + 1;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* FP32 formulation (fixed so a GPU kernel can be compared bit for bit).     */
/* With t = fma(x, x, cr) = x^2 + Re C:                                      */
/*   escape test   fma(y, y, t) > fl(4 + cr)   (|Z|^2 + Re C > 4 + Re C)     */
/*   Re Z'       = fma(-y, y, t)                                             */
/*   Im Z'       = fma(x + x, y, ci)                                         */
/* The test shares x^2 + Re C with the update; both of its sides carry Re C. */
/* Z_0 and C are the binary64 values rounded once to binary32.               */
/* ------------------------------------------------------------------------ */
static int32_t count_fp32(float x, float y, float cr, float ci, int32_t max_iter)
{
    const float lim = 4.0f + cr;
    int32_t n = 0;
    while (n < max_iter) {
        float t = fmaf(x, x, cr);
        float m = fmaf(y, y, t);
        if (m > lim)
            break;
        float xn = fmaf(-y, y, t);
        float tx = x + x;
        float yn = fmaf(tx, y, ci);
        x = xn;
        y = yn;
        n = n + 1;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Float-float ("double-single") arithmetic: a value is hi + lo with two     */
/* binary32 numbers, |lo| <= ulp(hi)/2.  Built from error-free transforms:   */
/*   TwoSum (Knuth; Moller): s = RN(a+b), e = (a+b) - s exactly.             */
/*   Fast2Sum (Dekker 1971): the same when |a| >= |b| or a == 0.             */
/*   TwoProd with FMA: p = RN(ab), e = fma(a, b, -p) = ab - p exactly.       */
/* Double-word sum and product follow Joldes, Muller and Popescu, "Tight and */
/* rigorous error bounds for basic building blocks of double-word            */
/* arithmetic" (ACM TOMS 2017): the accurate sum of two double-words         */
/* (relative error below 3u^2, also under cancellation, which x^2 - y^2      */
/* needs) and the FMA-based product of two double-words (below 4u^2).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    float hi, lo;
} dw;

void jro_two_sum(float a, float b, float *s, float *e)
{
    float sum = a + b;
    float b_part = sum - a;          /* what of b made it into sum */
    float a_part = sum - b_part;     /* what of a made it into sum */
    float a_err = a - a_part;
    float b_err = b - b_part;
    *s = sum;
    *e = a_err + b_err;
}

void jro_fast_two_sum(float a, float b, float *s, float *e)
{
    float sum = a + b;
    float b_part = sum - a;
    *s = sum;
    *e = b - b_part;
}

void jro_two_prod(float a, float b, float *p, float *e)
{
    float prod = a * b;
    *p = prod;
    *e = fmaf(a, b, -prod);
}

static dw dw_add(dw x, dw y)
{
    float sh, sl, th, tl, vh, vl;
    dw z;
    jro_two_sum(x.hi, y.hi, &sh, &sl);       /* high parts, exactly   */
    jro_two_sum(x.lo, y.lo, &th, &tl);       /* low parts, exactly    */
    float c = sl + th;
    jro_fast_two_sum(sh, c, &vh, &vl);       /* renormalise           */
    float w = tl + vl;
    jro_fast_two_sum(vh, w, &z.hi, &z.lo);   /* renormalise again     */
    return z;
}

static dw dw_mul(dw x, dw y)
{
    float ch, cl1;
    dw z;
    jro_two_prod(x.hi, y.hi, &ch, &cl1);     /* hi*hi, exactly        */
    float low_low = x.lo * y.lo;
    float cross1 = fmaf(x.hi, y.lo, low_low);
    float cross = fmaf(x.lo, y.hi, cross1);  /* hi*lo + lo*hi + lo*lo */
    float cl = cl1 + cross;
    jro_fast_two_sum(ch, cl, &z.hi, &z.lo);
    return z;
}

static dw dw_neg(dw x)
{
    dw z;
    z.hi = -x.hi;
    z.lo = -x.lo;
    return z;
}

static dw dw_twice(dw x)
{
    dw z;
    z.hi = 2.0f * x.hi; /* exact */
    z.lo = 2.0f * x.lo; /* exact */
    return z;
}

/* hi = RN32(v), lo = RN32(v - hi); v - hi is exact in binary64. */
static dw dw_from_double(double v)
{
    dw z;
    z.hi = (float)v;
    z.lo = (float)(v - (double)z.hi);
    return z;
}

void jro_dw_add(float xh, float xl, float yh, float yl, float *zh, float *zl)
{
    dw x = {xh, xl}, y = {yh, yl};
    dw z = dw_add(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

void jro_dw_mul(float xh, float xl, float yh, float yl, float *zh, float *zl)
{
    dw x = {xh, xl}, y = {yh, yl};
    dw z = dw_mul(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

void jro_dw_split(double v, float *hi, float *lo)
{
    dw z = dw_from_double(v);
    *hi = z.hi;
    *lo = z.lo;
}

/* Cheaper double-word operations of the quadratic map's float-float
 * formulation (the general maps keep dw_add and dw_mul):
 *   dw_sqr       the square: TwoProd of the high part, plus one fused
 *                2*hi*lo term (2*hi is exact); the lo*lo term, below u^2
 *                of the result, is left out; one Fast2Sum.
 *   dw_add_cheap the sum: TwoSum of the high parts, the low parts' sum
 *                added to its error, one Fast2Sum (the "sloppy" double-word
 *                sum of Joldes, Muller and Popescu): for operands of one sign
 *                its error stays below a few u^2 of the result; under
 *                cancellation it is bounded by u^2 of the operands. */
static dw dw_sqr(dw x)
{
    float p, e;
    jro_two_prod(x.hi, x.hi, &p, &e);
    float twice_hi = x.hi + x.hi;               /* exact */
    float q = fmaf(twice_hi, x.lo, e);
    dw z;
    jro_fast_two_sum(p, q, &z.hi, &z.lo);
    return z;
}

static dw dw_add_cheap(dw x, dw y)
{
    float sh, sl;
    jro_two_sum(x.hi, y.hi, &sh, &sl);
    float lows = x.lo + y.lo;
    float err = sl + lows;
    dw z;
    jro_fast_two_sum(sh, err, &z.hi, &z.lo);
    return z;
}

void jro_dw_sqr(float xh, float xl, float *zh, float *zl)
{
    dw x = {xh, xl};
    dw z = dw_sqr(x);
    *zh = z.hi;
    *zl = z.lo;
}

void jro_dw_add_cheap(float xh, float xl, float yh, float yl, float *zh, float *zl)
{
    dw x = {xh, xl}, y = {yh, yl};
    dw z = dw_add_cheap(x, y);
    *zh = z.hi;
    *zl = z.lo;
}

/* |Z|^2 <= 4 for a double-word m: hi < 4, or hi == 4 and lo <= 0. */
static int dw_not_above_four(dw m)
{
    return (m.hi < 4.0f) || (m.hi == 4.0f && m.lo <= 0.0f);
}

/* Float-float formulation of the same iteration:                           */
/*   x2 = sqr(x), y2 = sqr(y), |Z|^2 = x2 +' y2 (one sign: exact enough to    */
/*   decide |Z|^2 > 4 against the double-word 4),                           */
/*   Re Z' = (x2 +' (-y2)) +' cr,  Im Z' = ((2x) * y) +' ci,                  */
/* sqr the double-word square, * the double-word product, +' the cheaper     */
/* double-word sum (dw_add_cheap).                                           */
static int32_t count_ff(dw x, dw y, dw cr, dw ci, int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        dw x2 = dw_sqr(x);
        dw y2 = dw_sqr(y);
        dw m = dw_add_cheap(x2, y2);
        if (!dw_not_above_four(m))
            break;
        dw re = dw_add_cheap(x2, dw_neg(y2));
        dw xn = dw_add_cheap(re, cr);
        dw im = dw_mul(dw_twice(x), y);
        dw yn = dw_add_cheap(im, ci);
        x = xn;
        y = yn;
        n = n + 1;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* General maps Z^d + C (d = 2..8): Z^d by d - 1 complex products from Z.    */
/* ------------------------------------------------------------------------ */
static int32_t count_fp64_general(double x, double y, double cr, double ci, int32_t d,
                                  int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        double x2 = x * x;
        double y2 = y * y;
        double m = x2 + y2;
        if (m > 4.0)
            break;
        double wr = x, wi = y;
        for (int32_t k = 1; k < d; k++) {
            double p_rr = wr * x;  /* Re W Re Z */
            double p_ii = wi * y;  /* Im W Im Z */
            double p_ri = wr * y;  /* Re W Im Z */
            double p_ir = wi * x;  /* Im W Re Z */
            double nr = p_rr - p_ii;
            double ni = p_ri + p_ir;
            wr = nr;
            wi = ni;
        }
        x = wr + cr;
        y = wi + ci;
        n = n + 1;
    }
    return n;
}

static int32_t count_fp32_general(float x, float y, float cr, float ci, int32_t d,
                                  int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        float x2 = x * x;
        float y2 = y * y;
        float m = x2 + y2;
        if (m > 4.0f)
            break;
        float wr = x, wi = y;
        for (int32_t k = 1; k < d; k++) {
            float p_rr = wr * x;
            float p_ii = wi * y;
            float p_ri = wr * y;
            float p_ir = wi * x;
            float nr = p_rr - p_ii;
            float ni = p_ri + p_ir;
            wr = nr;
            wi = ni;
        }
        x = wr + cr;
        y = wi + ci;
        n = n + 1;
    }
    return n;
}

static int32_t count_ff_general(dw x, dw y, dw cr, dw ci, int32_t d, int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        dw m = dw_add(dw_mul(x, x), dw_mul(y, y));
        if (!dw_not_above_four(m))
            break;
        dw wr = x, wi = y;
        for (int32_t k = 1; k < d; k++) {
            dw p_rr = dw_mul(wr, x);
            dw p_ii = dw_mul(wi, y);
            dw p_ri = dw_mul(wr, y);
            dw p_ir = dw_mul(wi, x);
            dw nr = dw_add(p_rr, dw_neg(p_ii));
            dw ni = dw_add(p_ri, p_ir);
            wr = nr;
            wi = ni;
        }
        x = dw_add(wr, cr);
        y = dw_add(wi, ci);
        n = n + 1;
    }
    return n;
}

int32_t jro_count_general(int32_t dtype, int32_t degree, double x0, double y0,
                          double cr, double ci, int32_t max_iter)
{
    if (dtype == JRO_FP32)
        return count_fp32_general((float)x0, (float)y0, (float)cr, (float)ci, degree,
                                  max_iter);
    if (dtype == JRO_FF)
        return count_ff_general(dw_from_double(x0), dw_from_double(y0), dw_from_double(cr),
                                dw_from_double(ci), degree, max_iter);
    return count_fp64_general(x0, y0, cr, ci, degree, max_iter);
}

static int32_t pixel_count_general(int32_t dtype, int32_t mode, int32_t degree, double cr,
                                   double ci, double re_min, double re_max, double im_min,
                                   double im_max, int32_t W, int32_t H, int32_t max_iter,
                                   int32_t i, int32_t j)
{
    double x, y;
    jro_pixel_center(re_min, re_max, im_min, im_max, W, H, i, j, &x, &y);
    if (mode == JRO_MANDELBROT)
        return jro_count_general(dtype, degree, 0.0, 0.0, x, y, max_iter);
    return jro_count_general(dtype, degree, x, y, cr, ci, max_iter);
}

void jro_render_general(int32_t dtype, int32_t mode, int32_t degree, double cr, double ci,
                        double re_min, double re_max, double im_min, double im_max,
                        int32_t W, int32_t H, int32_t max_iter, int32_t *out)
{
    for (int32_t j = 0; j < H; j++)
        for (int32_t i = 0; i < W; i++)
            out[(int64_t)j * W + i] = pixel_count_general(dtype, mode, degree, cr, ci, re_min,
                                                          re_max, im_min, im_max, W, H,
                                                          max_iter, i, j);
}

void jro_render_pixels_general(int32_t dtype, int32_t mode, int32_t degree, double cr,
                               double ci, double re_min, double re_max, double im_min,
                               double im_max, int32_t W, int32_t H, int32_t max_iter,
                               int64_t n, const int32_t *ii, const int32_t *jj, int32_t *out)
{
    for (int64_t k = 0; k < n; k++)
        out[k] = pixel_count_general(dtype, mode, degree, cr, ci, re_min, re_max, im_min,
                                     im_max, W, H, max_iter, ii[k], jj[k]);
}

/* ------------------------------------------------------------------------ */
/* Rational maps with two parameters: Z^d + C + lambda / Z^d (d = 2..8).     */
/* W = Z^d by the general maps' products; lambda / W is                      */
/* ((lr wr + li wi) + i (li wr - lr wi)) / (wr wr + wi wi), each product,    */
/* sum and quotient rounded; then Z' = ((wr + cr) + tr) + i ((wi + ci) + ti).*/
/* The test is "escaped unless |Z|^2 <= 4", so an iterate that is not a     */
/* number (0 / 0 at the pole Z = 0) counts as escaped.                       */
/* ------------------------------------------------------------------------ */
static int32_t count_fp64_rational(double x, double y, double cr, double ci, double lr,
                                   double li, int32_t d, int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        double x2 = x * x;
        double y2 = y * y;
        double m = x2 + y2;
        if (!(m <= 4.0))
            break;
        double wr = x, wi = y;          /* W = Z^d, as for the general maps */
        for (int32_t k = 1; k < d; k++) {
            double u_rr = wr * x;
            double u_ii = wi * y;
            double u_ri = wr * y;
            double u_ir = wi * x;
            double vr = u_rr - u_ii;
            double vi = u_ri + u_ir;
            wr = vr;
            wi = vi;
        }
        double q_r = wr * wr;
        double q_i = wi * wi;
        double q = q_r + q_i;          /* |W|^2 */
        double a = lr * wr;
        double b = li * wi;
        double e = li * wr;
        double f = lr * wi;
        double num_r = a + b;          /* Re(lambda conj(W)) */
        double num_i = e - f;          /* Im(lambda conj(W)) */
        double tr = num_r / q;
        double ti = num_i / q;
        double sr = wr + cr;
        double si = wi + ci;
        x = sr + tr;
        y = si + ti;
        n = n + 1;
    }
    return n;
}

static int32_t count_fp32_rational(float x, float y, float cr, float ci, float lr, float li,
                                   int32_t d, int32_t max_iter)
{
    int32_t n = 0;
    while (n < max_iter) {
        float x2 = x * x;
        float y2 = y * y;
        float m = x2 + y2;
        if (!(m <= 4.0f))
            break;
        float wr = x, wi = y;          /* W = Z^d, as for the general maps */
        for (int32_t k = 1; k < d; k++) {
            float u_rr = wr * x;
            float u_ii = wi * y;
            float u_ri = wr * y;
            float u_ir = wi * x;
            float vr = u_rr - u_ii;
            float vi = u_ri + u_ir;
            wr = vr;
            wi = vi;
        }
        float q_r = wr * wr;
        float q_i = wi * wi;
        float q = q_r + q_i;
        float a = lr * wr;
        float b = li * wi;
        float e = li * wr;
        float f = lr * wi;
        float num_r = a + b;
        float num_i = e - f;
        float tr = num_r / q;
        float ti = num_i / q;
        float sr = wr + cr;
        float si = wi + ci;
        x = sr + tr;
        y = si + ti;
        n = n + 1;
    }
    return n;
}

int32_t jro_count_rational(int32_t dtype, int32_t degree, double x0, double y0, double cr,
                           double ci, double lr, double li, int32_t max_iter)
{
    if (dtype == JRO_FP32)
        return count_fp32_rational((float)x0, (float)y0, (float)cr, (float)ci, (float)lr,
                                   (float)li, degree, max_iter);
    return count_fp64_rational(x0, y0, cr, ci, lr, li, degree, max_iter);
}

void jro_render_rational(int32_t dtype, int32_t degree, double cr, double ci, double lr,
                         double li, double re_min, double re_max, double im_min,
                         double im_max, int32_t W, int32_t H, int32_t max_iter, int32_t *out)
{
    for (int32_t j = 0; j < H; j++)
        for (int32_t i = 0; i < W; i++) {
            double x, y;
            jro_pixel_center(re_min, re_max, im_min, im_max, W, H, i, j, &x, &y);
            out[(int64_t)j * W + i] = jro_count_rational(dtype, degree, x, y, cr, ci, lr, li,
                                                         max_iter);
        }
}

void jro_render_pixels_rational(int32_t dtype, int32_t degree, double cr, double ci,
                                double lr, double li, double re_min, double re_max,
                                double im_min, double im_max, int32_t W, int32_t H,
                                int32_t max_iter, int64_t n, const int32_t *ii,
                                const int32_t *jj, int32_t *out)
{
    for (int64_t k = 0; k < n; k++) {
        double x, y;
        jro_pixel_center(re_min, re_max, im_min, im_max, W, H, ii[k], jj[k], &x, &y);
        out[k] = jro_count_rational(dtype, degree, x, y, cr, ci, lr, li, max_iter);
    }
}

/* ------------------------------------------------------------------------ */
/* Prescribed parameter path (Section 3): constants on the cardioid          */
/*   f(t) = ((2 cos t - cos 2t) / a, (2 sin t - sin 2t) / a) = (2u - u^2) / a, */
/* u = e^{it}, with the cardioid growing along the path (a decreasing).      */
/* Frame k: u_k = step^k (step = e^{i dt}) by square-and-multiply over the   */
/* bits of k from the highest, a_k = a0 - da k, C_k = (2 u_k - u_k^2) / a_k; */
/* every product, sum and quotient rounded to binary64, no fused operation.  */
/* ------------------------------------------------------------------------ */
static void cmul(double a, double b, double c, double d, double *re, double *im)
{
    double ac = a * c;
    double bd = b * d;
    double ad = a * d;
    double bc = b * c;
    *re = ac - bd;
    *im = ad + bc;
}

void jro_cardioid_constant(double step_re, double step_im, double a0, double da, int32_t k,
                           double *cr, double *ci)
{
    double pr = 1.0, pi = 0.0;
    for (int32_t bit = 30; bit >= 0; bit--) {
        cmul(pr, pi, pr, pi, &pr, &pi);
        if ((k >> bit) & 1)
            cmul(pr, pi, step_re, step_im, &pr, &pi);
    }
    double wr, wi;
    cmul(pr, pi, pr, pi, &wr, &wi);        /* u^2 */
    double dk = da * (double)k;
    double a = a0 - dk;
    double nr = 2.0 * pr - wr;
    double ni = 2.0 * pi - wi;
    *cr = nr / a;
    *ci = ni / a;
}

/* ------------------------------------------------------------------------ */
/* One orbit in the chosen formulation.                                      */
/* ------------------------------------------------------------------------ */
int32_t jro_count(int32_t dtype, double x0, double y0, double cr, double ci,
                  int32_t max_iter)
{
    if (dtype == JRO_FP32)
        return count_fp32((float)x0, (float)y0, (float)cr, (float)ci, max_iter);
    if (dtype == JRO_FF)
        return count_ff(dw_from_double(x0), dw_from_double(y0),
                        dw_from_double(cr), dw_from_double(ci), max_iter);
    return count_fp64(x0, y0, cr, ci, max_iter);
}

static int32_t pixel_count(int32_t dtype, int32_t mode, double cr, double ci,
                           double re_min, double re_max, double im_min, double im_max,
                           int32_t W, int32_t H, int32_t max_iter, int32_t i, int32_t j)
{
    double x, y;
    jro_pixel_center(re_min, re_max, im_min, im_max, W, H, i, j, &x, &y);
    if (mode == JRO_MANDELBROT)
        return jro_count(dtype, 0.0, 0.0, x, y, max_iter); /* Z_0 = 0, C = pixel */
    return jro_count(dtype, x, y, cr, ci, max_iter);       /* Z_0 = pixel       */
}

/* ------------------------------------------------------------------------ */
/* Colour levels (Section 2): count k takes entry k of the table; counts    */
/* beyond its last entry take the last entry.                                */
/* ------------------------------------------------------------------------ */
void jro_colorize(const int32_t *counts, int64_t n, const uint32_t *palette,
                  int32_t palette_len, uint32_t *out)
{
    for (int64_t k = 0; k < n; k++) {
        int32_t level = counts[k];
        if (level > palette_len - 1)
            level = palette_len - 1;
        out[k] = palette[level];
    }
}

/* The sequential version of Section 2: one main loop over the pixel region. */
void jro_render(int32_t dtype, int32_t mode, double cr, double ci,
                double re_min, double re_max, double im_min, double im_max,
                int32_t W, int32_t H, int32_t max_iter, int32_t *out)
{
    for (int32_t j = 0; j < H; j++)
        for (int32_t i = 0; i < W; i++)
            out[(int64_t)j * W + i] = pixel_count(dtype, mode, cr, ci, re_min, re_max,
                                                  im_min, im_max, W, H, max_iter, i, j);
}

void jro_render_pixels(int32_t dtype, int32_t mode, double cr, double ci,
                       double re_min, double re_max, double im_min, double im_max,
                       int32_t W, int32_t H, int32_t max_iter, int64_t n,
                       const int32_t *ii, const int32_t *jj, int32_t *out)
{
    for (int64_t k = 0; k < n; k++)
        out[k] = pixel_count(dtype, mode, cr, ci, re_min, re_max, im_min, im_max,
                             W, H, max_iter, ii[k], jj[k]);
}
