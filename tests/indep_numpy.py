"""Second, independent implementations of the three arithmetic formulations.

Written separately from the C oracle (vectorised numpy, one ufunc per IEEE
operation) so that a bit-for-bit match between the two pins the oracle's
mapping, operation order and count convention.  numpy evaluates float32 and
float64 ufuncs in their own precision and never fuses a multiply with an add.

binary32 fused multiply-add is emulated exactly: the float64 product of two
float32 values is exact, the float64 sum is then rounded to odd (Boldo and
Melquiond, "Emulation of FMA and correctly rounded sums: proved algorithms
using rounding to odd", IEEE TC 2008) and rounded once more to float32, which
gives the correctly rounded fma because float64 carries more than 24 + 2 bits.
"""
import numpy as np

F32 = np.float32
F64 = np.float64


def pixel_grid(window, W, H):
    """binary64 pixel centres, x[j, i] and y[j, i]; row 0 is im_max."""
    re_min, re_max, im_min, im_max = (float(v) for v in window)
    hx = (re_max - re_min) / (2.0 * W)
    hy = (im_max - im_min) / (2.0 * H)
    cx = 0.5 * (re_min + re_max)
    cy = 0.5 * (im_min + im_max)
    oi = (2 * np.arange(W, dtype=np.int64) + 1 - W).astype(F64)
    oj = (2 * np.arange(H, dtype=np.int64) + 1 - H).astype(F64)
    xs = F64(cx) + oi * F64(hx)
    ys = F64(cy) - oj * F64(hy)
    x = np.broadcast_to(xs[None, :], (H, W)).copy()
    y = np.broadcast_to(ys[:, None], (H, W)).copy()
    return x, y


def fmaf(a, b, c):
    a = np.asarray(a, F32)
    b = np.asarray(b, F32)
    c = np.asarray(c, F32)
    p = a.astype(F64) * b.astype(F64)          # exact
    c64 = c.astype(F64)
    s = p + c64                                  # RN64
    bp = s - p                                   # TwoSum error of p + c
    ap = s - bp
    e = (p - ap) + (c64 - bp)
    bits = s.view(np.int64)
    fix = (e != 0) & ((bits & 1) == 0)           # inexact and even: go to odd neighbour
    toward = np.where(e > 0, np.inf, -np.inf)
    s = np.where(fix, np.nextafter(s, toward), s)
    return s.astype(F32)


def _iterate(state, step, escaped_fn, max_iter):
    """Generic per-pixel loop: counts[k] = first n with escaped, capped."""
    shape = escaped_fn(state).shape
    counts = np.zeros(shape, dtype=np.int32)
    active = np.ones(shape, dtype=bool)
    for n in range(max_iter):
        esc = escaped_fn(state) & active
        active &= ~esc
        if not active.any():
            break
        counts[active] += 1
        state = step(state, active)
    return counts


# ---------------------------------------------------------------- FP64
def counts_fp64(x0, y0, cr, ci, max_iter):
    x0 = np.asarray(x0, F64)
    y0 = np.asarray(y0, F64)
    cr = np.broadcast_to(np.asarray(cr, F64), x0.shape)
    ci = np.broadcast_to(np.asarray(ci, F64), x0.shape)

    def esc(s):
        x, y = s
        return (x * x + y * y) > 4.0

    def step(s, act):
        x, y = s
        xn = (x * x - y * y) + cr
        yn = ((2.0 * x) * y) + ci
        return (np.where(act, xn, x), np.where(act, yn, y))

    return _iterate((x0, y0), step, esc, max_iter)


# ---------------------------------------------------------------- FP32
def counts_fp32(x0, y0, cr, ci, max_iter):
    x0 = np.asarray(x0, F64).astype(F32)
    y0 = np.asarray(y0, F64).astype(F32)
    cr = np.broadcast_to(np.asarray(cr, F64).astype(F32), x0.shape)
    ci = np.broadcast_to(np.asarray(ci, F64).astype(F32), x0.shape)

    lim = F32(4.0) + cr

    def esc(s):
        x, y = s
        return fmaf(y, y, fmaf(x, x, cr)) > lim

    def step(s, act):
        x, y = s
        xn = fmaf(-y, y, fmaf(x, x, cr))
        yn = fmaf(x + x, y, ci)
        return (np.where(act, xn, x), np.where(act, yn, y))

    return _iterate((x0, y0), step, esc, max_iter)


# ---------------------------------------------------------------- float-float
def split(v):
    v = np.asarray(v, F64)
    hi = v.astype(F32)
    lo = (v - hi.astype(F64)).astype(F32)
    return hi, lo


def two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def fast_two_sum(a, b):
    s = a + b
    return s, b - (s - a)


def dw_add(x, y):
    sh, sl = two_sum(x[0], y[0])
    th, tl = two_sum(x[1], y[1])
    vh, vl = fast_two_sum(sh, sl + th)
    return fast_two_sum(vh, tl + vl)


def dw_mul(x, y):
    ch = x[0] * y[0]
    cl1 = fmaf(x[0], y[0], -ch)
    t = fmaf(x[1], y[0], fmaf(x[0], y[1], x[1] * y[1]))
    return fast_two_sum(ch, cl1 + t)


def dw_sqr(x):
    """h^2 exactly as p + e, then 2 h l fused onto e; l^2 left out."""
    p = x[0] * x[0]
    e = fmaf(x[0], x[0], -p)
    return fast_two_sum(p, fmaf(x[0] * F32(2), x[1], e))


def dw_add_cheap(x, y):
    """TwoSum of the high words; the low words' sum joins its error."""
    sh, sl = two_sum(x[0], y[0])
    return fast_two_sum(sh, sl + (x[1] + y[1]))


def counts_ff(x0, y0, cr, ci, max_iter):
    shape = np.shape(x0)
    x = split(x0)
    y = split(y0)
    crs = tuple(np.broadcast_to(a, shape) for a in split(cr))
    cis = tuple(np.broadcast_to(a, shape) for a in split(ci))

    def esc(s):
        xx, yy = s
        m = dw_add_cheap(dw_sqr(xx), dw_sqr(yy))
        return ~((m[0] < 4) | ((m[0] == 4) & (m[1] <= 0)))

    def step(s, act):
        xx, yy = s
        x2 = dw_sqr(xx)
        y2 = dw_sqr(yy)
        xn = dw_add_cheap(dw_add_cheap(x2, (-y2[0], -y2[1])), crs)
        yn = dw_add_cheap(dw_mul((xx[0] * F32(2), xx[1] * F32(2)), yy), cis)
        pick = lambda new, old: (np.where(act, new[0], old[0]), np.where(act, new[1], old[1]))
        return (pick(xn, xx), pick(yn, yy))

    with np.errstate(over="ignore", invalid="ignore"):
        return _iterate((x, y), step, esc, max_iter)


# ------------------------------------------------------ general maps Z^d + C
def _power_add(x, y, d, mul, sub, add, cr, ci):
    """Z^d by d - 1 products W <- W Z from W = Z, then + C."""
    wr, wi = x, y
    for _ in range(d - 1):
        nr = sub(mul(wr, x), mul(wi, y))
        ni = add(mul(wr, y), mul(wi, x))
        wr, wi = nr, ni
    return add(wr, cr), add(wi, ci)


def counts_general(x0, y0, cr, ci, max_iter, degree, dtype):
    if dtype == "ff":
        shape = np.shape(x0)
        x, y = split(x0), split(y0)
        crs = tuple(np.broadcast_to(a, shape) for a in split(cr))
        cis = tuple(np.broadcast_to(a, shape) for a in split(ci))
        neg = lambda a: (-a[0], -a[1])

        def esc(s):
            xx, yy = s
            m = dw_add(dw_mul(xx, xx), dw_mul(yy, yy))
            return ~((m[0] < 4) | ((m[0] == 4) & (m[1] <= 0)))

        def step(s, act):
            xx, yy = s
            xn, yn = _power_add(xx, yy, degree, dw_mul, lambda a, b: dw_add(a, neg(b)), dw_add,
                                crs, cis)
            pick = lambda new, old: (np.where(act, new[0], old[0]), np.where(act, new[1], old[1]))
            return (pick(xn, xx), pick(yn, yy))

        with np.errstate(over="ignore", invalid="ignore"):
            return _iterate((x, y), step, esc, max_iter)
    T = F32 if dtype == "fp32" else F64
    x0 = np.asarray(x0, F64).astype(T)
    y0 = np.asarray(y0, F64).astype(T)
    cr = np.broadcast_to(np.asarray(cr, F64).astype(T), x0.shape)
    ci = np.broadcast_to(np.asarray(ci, F64).astype(T), x0.shape)

    def esc(s):
        x, y = s
        return (x * x + y * y) > T(4.0)

    def step(s, act):
        x, y = s
        xn, yn = _power_add(x, y, degree, np.multiply, np.subtract, np.add, cr, ci)
        return (np.where(act, xn, x), np.where(act, yn, y))

    with np.errstate(over="ignore", invalid="ignore"):
        return _iterate((x0, y0), step, esc, max_iter)


def render_general(c, window, W, H, max_iter, dtype="fp64", mode="julia", degree=3):
    x, y = pixel_grid(window, W, H)
    c = complex(c)
    if mode == "mandelbrot":
        z = np.zeros_like(x)
        return counts_general(z, z, x, y, max_iter, degree, dtype)
    return counts_general(x, y, c.real, c.imag, max_iter, degree, dtype)


def counts_rational(x0, y0, cr, ci, lr, li, max_iter, degree, dtype):
    """The two-parameter rational map Z^d + C + lam / Z^d, one ufunc per
    rounded operation: W = Z^d as in _power_add, lam / W = (lam conj W) /
    |W|^2 in real arithmetic (numpy's own complex division uses another
    algorithm), then (W + C) + lam / W.  An iterate that is not a number
    counts as escaped (the test is "not |Z|^2 <= 4")."""
    T = F32 if dtype == "fp32" else F64
    x0 = np.asarray(x0, F64).astype(T)
    y0 = np.asarray(y0, F64).astype(T)
    cr, ci, lr, li = (np.broadcast_to(np.asarray(v, F64).astype(T), x0.shape)
                      for v in (cr, ci, lr, li))

    def esc(s):
        x, y = s
        return ~((x * x + y * y) <= T(4.0))

    def step(s, act):
        x, y = s
        wr, wi = x, y
        for _ in range(degree - 1):
            wr, wi = wr * x - wi * y, wr * y + wi * x
        q = wr * wr + wi * wi
        xn = (wr + cr) + (lr * wr + li * wi) / q
        yn = (wi + ci) + (li * wr - lr * wi) / q
        return (np.where(act, xn, x), np.where(act, yn, y))

    with np.errstate(all="ignore"):
        return _iterate((x0, y0), step, esc, max_iter)


def render_rational(c, lam, window, W, H, max_iter, dtype="fp64", degree=2):
    x, y = pixel_grid(window, W, H)
    c, lam = complex(c), complex(lam)
    return counts_rational(x, y, c.real, c.imag, lam.real, lam.imag, max_iter, degree, dtype)


COUNTS = {"fp64": counts_fp64, "fp32": counts_fp32, "ff": counts_ff}


def render(c, window, W, H, max_iter, dtype="fp64", mode="julia"):
    x, y = pixel_grid(window, W, H)
    c = complex(c)
    fn = COUNTS[dtype]
    if mode == "mandelbrot":
        z = np.zeros_like(x)
        return fn(z, z, x, y, max_iter)
    return fn(x, y, c.real, c.imag, max_iter)
