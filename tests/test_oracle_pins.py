"""Pins of the CPU oracle against what the paper and the mathematics fix.

Method: Mayfield et al., Section 2 (escape-time iteration of Z^2 + C over
pixels scaled onto the complex plane, iteration cap) and Section 3 (Mandelbrot
variant with Z_0 = 0, main cardioid border f(t) with a = 4).  None of these
checks reuses the oracle's own code: expected values come from hand-derived
orbits, closed forms, symmetries of the map, exact rational or high-precision
arithmetic, and a second numpy implementation written separately.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import indep_numpy as ind

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DTYPES = ("fp64", "fp32", "ff")
UNIT = (-1.5, 1.5, -1.5, 1.5)
C1 = complex(-0.8, 0.156)


def read_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------ orbits
@pytest.mark.parametrize("dtype", DTYPES)
def test_exact_small_orbits(dtype):
    rows = read_table("exact_orbits.txt")
    assert len(rows) >= 15
    for zr, zi, cr, ci, cnt in rows:
        z0 = complex(float(zr), float(zi))
        c = complex(float(cr), float(ci))
        for cap in (0, 1, 2, 5, 100, 1000):
            want = cap if cnt == "cap" else min(int(cnt), cap)
            got = oracle.count(z0, c, cap, dtype)
            assert got == want, (dtype, z0, c, cap, got, want)


def test_escape_by_less_than_fp32_ulp():
    """Z_0 = 2 + 2^-30, C = 0: |Z_0|^2 = 4 + 2^-28 + 2^-60 > 4, so the true count is 0.
    binary64 and float-float (hi = 2, lo = 2^-30) keep the excess; binary32
    rounds Z_0 to 2, where |Z_0|^2 = 4 is not > 4 and the orbit 2 -> 4 gives 1."""
    z0 = complex(2.0 + 2.0 ** -30, 0.0)
    assert oracle.count(z0, 0j, 100, "fp64") == 0
    assert oracle.count(z0, 0j, 100, "ff") == 0
    assert oracle.count(z0, 0j, 100, "fp32") == 1
    # just below: 2 - 2^-30 squares to 4 - 2^-28 + 2^-60 < 4, then 16 - ... > 4
    z1 = complex(2.0 - 2.0 ** -30, 0.0)
    assert oracle.count(z1, 0j, 100, "fp64") == 1
    assert oracle.count(z1, 0j, 100, "ff") == 1


def _rn32(q):
    """Round a rational to the nearest binary32 (ties to even); normal range."""
    from fractions import Fraction as Fr
    if q == 0:
        return Fr(0)
    sign = -1 if q < 0 else 1
    q = abs(q)
    e = q.numerator.bit_length() - q.denominator.bit_length()
    while Fr(2) ** e > q:
        e -= 1
    while Fr(2) ** (e + 1) <= q:
        e += 1
    scale = Fr(2) ** (23 - e)
    m = q * scale
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and lo % 2 == 1):
        lo += 1
    return sign * Fr(lo) / scale


def test_fp32_escape_test_formulation():
    """The FP32 formulation tests fma(y, y, fma(x, x, cr)) > fl(4 + cr): two
    single roundings of x^2 + cr and then + y^2, against 4 + cr rounded once.
    Points near |Z| = 2 where this decision differs from the plain
    RN(RN(x^2) + RN(y^2)) > 4 pin the formulation (expected values from exact
    rational arithmetic)."""
    rng = np.random.default_rng(11)
    found = 0
    for cr in (-0.8, 0.285, -1.75):
        crf = Fraction(float(np.float32(cr)))
        lim = _rn32(4 + crf)
        for _ in range(100000):
            t = rng.uniform(0, np.pi / 2)
            x = np.float32(2 * np.cos(t))
            y = np.float32(2 * np.sin(t))
            X, Y = Fraction(float(x)), Fraction(float(y))
            m = _rn32(Y * Y + _rn32(X * X + crf))
            ours = m > lim
            other = _rn32(_rn32(X * X) + _rn32(Y * Y)) > 4
            if ours != other:
                got = oracle.count(complex(float(x), float(y)), complex(cr, 0.0), 1, "fp32")
                assert got == (0 if ours else 1), (cr, x, y)
                found += 1
                if found % 4 == 0:
                    break
    assert found >= 8


# --------------------------------------------------- independent reimplementations
CASES = [
    # c, window, W, H, cap, mode
    (C1, UNIT, 512, 512, 100, "julia"),
    (complex(0.285, 0.01), (-1.3, 1.1, -0.7, 0.95), 97, 61, 250, "julia"),
    (complex(-0.4, 0.6), (-1.6, 1.6, -1.6, 1.6), 130, 257, 1000, "julia"),
    (0j, (-2.0, 1.0, -1.0, 1.3), 211, 173, 200, "mandelbrot"),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", DTYPES)
def test_matches_numpy_reimplementation(dtype, case):
    c, win, W, H, cap, mode = CASES[case]
    if dtype == "ff":  # the numpy float-float loop is slow; shrink the grid
        W, H = min(W, 120), min(H, 90)
    a = oracle.render(c, win, W, H, cap, dtype, mode)
    b = ind.render(c, win, W, H, cap, dtype, mode)
    assert a.shape == (H, W)
    np.testing.assert_array_equal(a, b)


def test_c1_fingerprint():
    """Single 512x512 image at C = -0.8+0.156i, window [-1.5,1.5]^2, cap 100.

    The numbers are those the numpy reimplementation gives (checked bit for bit
    above); here they guard the mapping of pixel (row, column) positions.
    """
    a = oracle.render(C1, UNIT, 512, 512, 100)
    assert int(a.sum()) == 4120640
    assert a[0, 0] == 0 and a[256, 256] == 100
    hist = np.bincount(a.ravel(), minlength=101)
    assert (hist[0], hist[1], hist[2], hist[3], hist[100]) == (1756, 92720, 52052, 24210, 23168)


def _py_count(x, y, cr, ci, cap):
    n = 0
    while n < cap:
        x2, y2 = x * x, y * y
        if x2 + y2 > 4.0:
            break
        x, y = (x2 - y2) + cr, ((2.0 * x) * y) + ci
        n += 1
    return n


def test_pure_python_definition():
    W, H, cap = 16, 12, 60
    win = (-1.7, 1.3, -1.1, 0.9)
    a = oracle.render(C1, win, W, H, cap)
    re_min, re_max, im_min, im_max = win
    hx, hy = (re_max - re_min) / (2.0 * W), (im_max - im_min) / (2.0 * H)
    cx, cy = 0.5 * (re_min + re_max), 0.5 * (im_min + im_max)
    for j in range(H):
        for i in range(W):
            x = cx + float(2 * i + 1 - W) * hx
            y = cy - float(2 * j + 1 - H) * hy
            assert a[j, i] == _py_count(x, y, C1.real, C1.imag, cap)


def test_pixel_centres():
    win = (-2.0, 2.0, -1.0, 3.0)
    x, y = oracle.pixel_center(win, 4, 2, 0, 0)
    assert (x, y) == (-1.5, 2.0)            # first column centre, top row centre
    x, y = oracle.pixel_center(win, 4, 2, 3, 1)
    assert (x, y) == (1.5, 0.0)
    x, y = oracle.pixel_center((-1.0, 1.0, -1.0, 1.0), 3, 3, 1, 1)
    assert (x, y) == (0.0, 0.0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_cap_zero_and_one(dtype):
    assert not oracle.render(C1, UNIT, 33, 17, 0, dtype).any()
    a1 = oracle.render(C1, UNIT, 33, 17, 1, dtype)
    assert set(np.unique(a1)) <= {0, 1}


# ------------------------------------------------------------ closed forms
def _c0_expected(z, cap):
    """C = 0: |Z_n| = |Z_0|^(2^n); count = cap iff |Z_0| <= 1, else the first n
    with |Z_0|^(2^n) > 2, i.e. 2^n log2|Z_0| > 1.  Returns (count, margin ok)."""
    r = abs(z)
    if r <= 1.0:
        return cap, True
    L = math.log2(r)
    n = 0
    while not (2.0 ** n * L > 1.0):
        n += 1
    return min(n, cap), n


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-13), ("fp32", 1e-5), ("ff", 1e-11)])
def test_closed_form_c_zero(dtype, tol):
    W = H = 64
    win = (-2.3, 2.3, -2.3, 2.3)
    cap = 40
    a = oracle.render(0j, win, W, H, cap, dtype)
    checked = 0
    for j in range(H):
        for i in range(W):
            x, y = oracle.pixel_center(win, W, H, i, j)
            if dtype == "fp32":
                x, y = float(np.float32(x)), float(np.float32(y))
            z = complex(x, y)
            r = abs(z)
            if abs(r - 1.0) < 1e-3:
                continue  # near the unit circle rounding walks the modulus
            want, n = _c0_expected(z, cap)
            if r > 1.0:
                L = math.log2(r)
                # skip pixels whose escape step sits within rounding of 2^n L = 1
                if any(abs(2.0 ** k * L - 1.0) < 2.0 ** k * tol for k in (n - 1, n) if k >= 0):
                    continue
            assert a[j, i] == want, (dtype, i, j, z, a[j, i], want)
            checked += 1
    assert checked > 0.95 * W * H


@pytest.mark.parametrize("dtype", DTYPES)
def test_c_minus_two_real_segment(dtype):
    """C = -2: real x in [-2, 2] gives x^2 - 2 in [-2, 2]; no real point of the
    segment ever escapes, and |Z|^2 = 4 at the ends pins the strict test."""
    W, H, cap = 401, 3, 500
    win = (-2.0 - 2.0 / 400, 2.0 + 2.0 / 400, -0.01, 0.01)  # centres hit -2 and 2
    a = oracle.render(complex(-2.0, 0.0), win, W, H, cap, dtype)
    x0, y0 = oracle.pixel_center(win, W, H, 0, 1)
    xe, _ = oracle.pixel_center(win, W, H, W - 1, 1)
    assert y0 == 0.0 and x0 == -2.0 and xe == 2.0
    assert (a[1] == cap).all()
    # off the segment, C = -2 is the Chebyshev map: Z = w + 1/w, Z_n = w^(2^n) + w^-(2^n)
    for w in (1.3 * np.exp(0.7j), 1.05 * np.exp(2.0j), 2.0 * np.exp(-1.1j), 1.01 * np.exp(0.3j)):
        z0 = complex(w + 1 / w)
        n = 0
        while abs(w ** (2 ** n) + w ** (-(2 ** n))) ** 2 <= 4.0 and n < cap:
            n += 1
        got = oracle.count(z0, -2.0, cap, dtype)
        assert abs(got - n) <= 1, (w, got, n)


# ------------------------------------------------------------- symmetries
@pytest.mark.parametrize("dtype", DTYPES)
def test_symmetries(dtype):
    W, H, cap = 96, 72, 150
    win = (-1.6, 1.6, -1.2, 1.2)
    c = complex(-0.123, 0.745)
    a = oracle.render(c, win, W, H, cap, dtype)
    # Z -> -Z: (-Z)^2 = Z^2, and the centred grid is exactly antisymmetric
    np.testing.assert_array_equal(a, a[::-1, ::-1])
    # conj(C) gives the conjugate orbit: the image flips top to bottom
    b = oracle.render(c.conjugate(), win, W, H, cap, dtype)
    np.testing.assert_array_equal(b, a[::-1, :])
    # real C: the image is its own mirror
    r = oracle.render(complex(-0.75, 0.0), win, W, H, cap, dtype)
    np.testing.assert_array_equal(r, r[::-1, :])
    # Mandelbrot image is symmetric under conjugation of C
    m = oracle.render(0j, (-2.0, 0.7, -1.2, 1.2), W + 1, H + 1, cap, dtype, "mandelbrot")
    np.testing.assert_array_equal(m, m[::-1, :])


# ------------------------------------------------- interiors (Sections 3, 4)
@pytest.mark.parametrize("dtype", DTYPES)
def test_main_cardioid_and_period2_bulb(dtype):
    """C = mu/2 - mu^2/4 with |mu| < 1 lies inside the main cardioid (its border
    is the a = 4 curve of Section 3): the fixed point mu/2 attracts, so the
    Mandelbrot orbit from 0 and the Julia orbit from mu/2 stay bounded.  For
    |C + 1| < 1/4 (the period-2 bulb, Section 4's bulbs and orbits) the orbit
    from 0 is bounded too."""
    rng = np.random.default_rng(7)
    cap = 400
    for _ in range(60):
        mu = 0.9 * np.sqrt(rng.uniform()) * np.exp(2j * np.pi * rng.uniform())
        c = complex(mu / 2 - mu * mu / 4)
        assert oracle.count(0j, c, cap, dtype) == cap
        assert oracle.count(complex(mu / 2), c, cap, dtype) == cap
        b = complex(-1.0 + 0.2 * np.sqrt(rng.uniform()) * np.exp(2j * np.pi * rng.uniform()))
        assert oracle.count(0j, b, cap, dtype) == cap


def test_paper_constants_on_cardioid_path():
    """Figure 2's constants are taken along f(t) with a = 3.9 (Section 3), just
    outside the main cardioid: |1 - sqrt(1 - 4C)| >= 1 there."""
    from workloads import cardioid_point
    rows = {r[0]: complex(float(r[1]), float(r[2])) for r in read_table("paper_constants.txt")}
    ts = np.linspace(0, 2 * np.pi, 200001)
    curve = np.array([cardioid_point(t, 3.9) for t in ts[::10]])
    for k in ("fig2_a", "fig2_b", "fig2_c", "fig2_d"):
        c = rows[k]
        d = np.min(np.abs(curve - c))
        assert d < 1e-3, (k, d)
        assert abs(1 - np.sqrt(1 - 4 * c)) >= 1.0, k
    # a = 4 traces the main cardioid border: multiplier |1 - sqrt(1 - 4C)| = 1
    for t in np.linspace(0.1, 6.2, 17):
        c = cardioid_point(t, 4.0)
        assert abs(abs(1 - np.sqrt(1 - 4 * c)) - 1.0) < 1e-12


# ------------------------------------------------ exact and high precision
def _exact_count(x0, y0, cr, ci, cap):
    x, y = Fraction(x0), Fraction(y0)
    cr, ci = Fraction(cr), Fraction(ci)
    n = 0
    while n < cap:
        if x * x + y * y > 4:
            break
        x, y = x * x - y * y + cr, 2 * x * y + ci
        n += 1
    return n


def test_exact_rational_counts_small_cap():
    """Exact rational arithmetic for caps <= 6; the binary64 oracle must agree on
    every pixel whose exact |Z_n|^2 keeps clear of 4 (all of them here)."""
    W, H, cap = 8, 8, 6
    win = (-1.5, 1.5, -1.5, 1.5)
    for c in (C1, complex(0.25, 0.5), complex(-1.0, 0.25)):
        a = oracle.render(c, win, W, H, cap)
        for j in range(H):
            for i in range(W):
                x, y = oracle.pixel_center(win, W, H, i, j)
                assert a[j, i] == _exact_count(x, y, c.real, c.imag, cap), (c, i, j)


def test_mpmath_brute_force():
    """High-precision orbits (64 + 2 cap bits: rounding error grows at most 4x
    per step while |Z| <= 2) decide the true count; binary64 must agree on each
    pixel whose orbit keeps |Z_n|^2 farther than 4^n * 2^-44 from 4."""
    mp = pytest.importorskip("mpmath")
    cap = 30
    mp.mp.prec = 64 + 2 * cap
    checked = 0
    for c, win in ((C1, UNIT), (complex(-0.4, 0.6), (-1.2, 1.2, -1.2, 1.2)),
                   (complex(0.285, 0.013), (-0.9, 0.3, -0.2, 1.0))):
        a = oracle.render(c, win, 8, 8, cap)
        cr, ci = mp.mpf(c.real), mp.mpf(c.imag)
        for j in range(8):
            for i in range(8):
                x0, y0 = oracle.pixel_center(win, 8, 8, i, j)
                x, y = mp.mpf(x0), mp.mpf(y0)
                n, clear = 0, True
                while n < cap:
                    m = x * x + y * y
                    if abs(m - 4) < mp.mpf(4) ** n * mp.mpf(2) ** -44:
                        clear = False
                    if m > 4:
                        break
                    x, y = x * x - y * y + cr, 2 * x * y + ci
                    n += 1
                if clear:
                    assert a[j, i] == n, (c, i, j, a[j, i], n)
                    checked += 1
    assert checked >= 100


# --------------------------------------------------- float-float primitives
def _f32(v):
    return float(np.float32(v))


def _rand_f32(rng, n, lo=-30, hi=30):
    m = rng.uniform(-1, 1, n)
    e = rng.integers(lo, hi, n)
    return [_f32(a * 2.0 ** b) for a, b in zip(m, e)]


def test_error_free_transforms():
    rng = np.random.default_rng(3)
    A = _rand_f32(rng, 3000, -10, 10)
    B = _rand_f32(rng, 3000, -10, 10)
    for a, b in zip(A, B):
        s, e = oracle.two_sum(a, b)
        assert s == _f32(a + b)
        assert Fraction(s) + Fraction(e) == Fraction(a) + Fraction(b)
        hi, lo = (a, b) if abs(a) >= abs(b) else (b, a)
        s2, e2 = oracle.fast_two_sum(hi, lo)
        assert Fraction(s2) + Fraction(e2) == Fraction(a) + Fraction(b)
        p, pe = oracle.two_prod(a, b)
        assert Fraction(p) + Fraction(pe) == Fraction(a) * Fraction(b)


def _dw(rng):
    hi = _f32(rng.uniform(-3, 3))
    lo = _f32(hi * 2.0 ** -24 * rng.uniform(-0.5, 0.5))
    s, e = oracle.fast_two_sum(hi, lo)  # normalise
    return s, e


def test_double_word_error_bounds():
    """Relative error below 3u^2 (sum, also under cancellation) and 4u^2
    (product), u = 2^-24, and the result is normalised."""
    rng = np.random.default_rng(5)
    u = Fraction(1, 2 ** 24)
    for _ in range(3000):
        x, y = _dw(rng), _dw(rng)
        if rng.uniform() < 0.3:  # force heavy cancellation in the sum
            y = (-x[0], _f32(-x[1] + x[0] * 2.0 ** -30 * rng.uniform(-1, 1)))
        X = Fraction(x[0]) + Fraction(x[1])
        Y = Fraction(y[0]) + Fraction(y[1])
        zh, zl = oracle.dw_add(x, y)
        if X + Y != 0:
            assert abs(Fraction(zh) + Fraction(zl) - (X + Y)) <= 3 * u * u * abs(X + Y)
        assert zh == _f32(zh + zl)
        ph, pl = oracle.dw_mul(x, y)
        if X * Y != 0:
            assert abs(Fraction(ph) + Fraction(pl) - X * Y) <= 4 * u * u * abs(X * Y)
        assert ph == _f32(ph + pl)


def test_cheap_double_word_error_bounds():
    """The quadratic map's float-float square and sum.  Square: relative
    error below 4u^2 (3u^2 from rounding h^2's error plus 2hl, u^2 from the
    dropped l^2).  Sum: relative error below 3u^2 for operands of one sign;
    under cancellation the error stays below 3u^2 of |x| + |y| (an absolute
    bound: the relative one is lost there).  Results normalised."""
    rng = np.random.default_rng(6)
    u = Fraction(1, 2 ** 24)
    for _ in range(3000):
        x, y = _dw(rng), _dw(rng)
        X = Fraction(x[0]) + Fraction(x[1])
        sh, sl = oracle.dw_sqr(x)
        assert abs(Fraction(sh) + Fraction(sl) - X * X) <= 4 * u * u * X * X
        assert sh == _f32(sh + sl)
        if rng.uniform() < 0.3:  # heavy cancellation
            y = (-x[0], _f32(-x[1] + x[0] * 2.0 ** -30 * rng.uniform(-1, 1)))
        elif rng.uniform() < 0.5:  # one sign
            if (x[0] > 0) != (y[0] > 0):
                y = (-y[0], -y[1])
        Y = Fraction(y[0]) + Fraction(y[1])
        zh, zl = oracle.dw_add_cheap(x, y)
        err = abs(Fraction(zh) + Fraction(zl) - (X + Y))
        if X * Y > 0:
            assert err <= 3 * u * u * abs(X + Y)
        assert err <= 3 * u * u * (abs(X) + abs(Y))
        assert zh == _f32(zh + zl)


def test_split():
    rng = np.random.default_rng(9)
    for v in rng.uniform(-2, 2, 500):
        hi, lo = oracle.dw_split(v)
        assert hi == _f32(v)
        assert abs(Fraction(hi) + Fraction(lo) - Fraction(v)) <= abs(Fraction(v)) * Fraction(1, 2 ** 47)


# -------------------------------------------- reduced precision vs FP64
@pytest.mark.parametrize("dtype,bound", [("fp32", 0.005), ("ff", 0.005)])
def test_mismatch_fraction_unit_window(dtype, bound):
    """At unit-scale windows with cap 100 the FP32 and float-float counts differ
    from binary64 on at most 0.5% of the pixels."""
    W = H = 256 if dtype == "fp32" else 128
    ref = oracle.render(C1, UNIT, W, H, 100, "fp64")
    got = oracle.render(C1, UNIT, W, H, 100, dtype)
    frac = float((ref != got).mean())
    assert frac <= bound, frac


# ------------------------------------------------ colour levels (Section 2)
def test_colorize_literal_table():
    """Count k takes entry k of the table; counts past its end take the last
    entry; a one-entry table paints everything."""
    counts = np.array([[0, 1, 2], [3, 4, 100]], dtype=np.int32)
    pal = np.array([0xFF000000, 0xFF0000FF, 0xFF00FF00, 0xFFFF0000], dtype=np.uint32)
    want = np.array([[0xFF000000, 0xFF0000FF, 0xFF00FF00],
                     [0xFFFF0000, 0xFFFF0000, 0xFFFF0000]], dtype=np.uint32)
    got = oracle.colorize(counts, pal)
    assert got.dtype == np.uint32 and got.shape == counts.shape
    np.testing.assert_array_equal(got, want)
    one = oracle.colorize(counts, np.array([0xDEADBEEF], dtype=np.uint32))
    assert (one == 0xDEADBEEF).all()


def test_colorize_identity_table_gives_the_counts():
    """Entry k = k over 0..cap returns the count image itself."""
    a = oracle.render(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 96, 80, 100)
    got = oracle.colorize(a, np.arange(101, dtype=np.uint32))
    np.testing.assert_array_equal(got.astype(np.int64), a.astype(np.int64))


def test_colorize_two_levels_mark_the_bounded_set():
    """A table that is 0 below the cap and all ones at the cap marks the
    bounded pixels.  For C = 0 they are exactly the closed unit disc; a
    Mandelbrot window inside the main cardioid is bounded everywhere."""
    cap = 60
    pal = np.zeros(cap + 1, dtype=np.uint32)
    pal[cap] = 0xFFFFFFFF
    W = H = 64
    win = (-1.7, 1.7, -1.7, 1.7)
    img = oracle.colorize(oracle.render(0j, win, W, H, cap), pal)
    checked = 0
    for j in range(H):
        for i in range(W):
            r = abs(complex(*oracle.pixel_center(win, W, H, i, j)))
            if abs(r - 1.0) < 1e-3:
                continue
            assert (img[j, i] == 0xFFFFFFFF) == (r <= 1.0), (i, j, r)
            checked += 1
    assert checked > 0.95 * W * H
    mwin = (-0.3, 0.15, -0.25, 0.25)
    for j in range(0, 33, 4):
        for i in range(0, 41, 4):
            c = complex(*oracle.pixel_center(mwin, 41, 33, i, j))
            mu = 1.0 - np.sqrt(1.0 - 4.0 * c + 0j)  # c = mu/2 - mu^2/4
            assert abs(mu) < 0.95
    m = oracle.colorize(oracle.render(0j, mwin, 41, 33, cap, "fp64", "mandelbrot"), pal)
    assert (m == 0xFFFFFFFF).all()


# ------------------------------------------- general maps Z^d + C (Section 4)
# Orbits of small integers and units: every value is exact in every
# precision, so the counts are those of exact arithmetic.
GENERAL_ORBITS = [
    # degree, Z_0, C, count (cap 100)
    (3, 0, 1, 3),        # 0, 1, 2 (|2|^2 = 4 is not > 4), 9
    (3, 0, -1, 3),       # 0, -1, -2, -9
    (4, 0, 1j, 3),       # 0, i, 1 + i, -4 + i
    (3, 2, 0, 1),        # 2 is not escaped, 8 is
    (3, 0, -2, 2),       # 0, -2, -10
    (5, 0, 2, 2),        # 0, 2, 34
    (3, 3, 0, 0),
    (4, 0, -1, 100),     # 0, -1, 0, -1, ...
    (3, 1j, 0, 100),     # i, -i, i, ...
    (6, -1, 0, 100),     # -1, 1, 1, ...
    (8, 0, 0, 100),
]


@pytest.mark.parametrize("dtype", DTYPES)
def test_general_exact_small_orbits(dtype):
    for d, z0, c, want in GENERAL_ORBITS:
        assert oracle.count(z0, c, 100, dtype, degree=d) == want, (d, z0, c)
        assert oracle.count(z0, c, 1, dtype, degree=d) == min(want, 1)
        assert oracle.count(z0, c, 0, dtype, degree=d) == 0


def test_general_degree_two_is_the_quadratic_map_fp64():
    """(a + ib)^2 by the general product is (a a - b b) + i (a b + b a), and
    a b + b a = 2 fl(a b) = fl((2a) b) when a b is normal: the general FP64
    formulation at d = 2 gives the quadratic FP64 counts bit for bit."""
    for c, win, mode in ((C1, (-1.5, 1.5, -1.5, 1.5), "julia"),
                         (complex(0.285, 0.01), (-1.2, 1.2, -0.9, 0.9), "julia"),
                         (0j, (-2.0, 0.6, -1.1, 1.1), "mandelbrot")):
        a = oracle.render_general(c, win, 64, 48, 300, "fp64", mode, 2)
        b = oracle.render(c, win, 64, 48, 300, "fp64", mode)
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("degree", [2, 3, 4, 5, 8])
def test_general_matches_numpy_reimplementation(dtype, degree):
    for c, win, mode in ((complex(0.4, 0.3), (-1.3, 1.3, -1.2, 1.2), "julia"),
                         (0j, (-1.5, 1.5, -1.5, 1.5), "mandelbrot")):
        a = oracle.render(c, win, 37, 29, 60, dtype, mode, degree) if degree > 2 else \
            oracle.render_general(c, win, 37, 29, 60, dtype, mode, degree)
        b = ind.render_general(c, win, 37, 29, 60, dtype, mode, degree)
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-12), ("fp32", 1e-4), ("ff", 1e-10)])
@pytest.mark.parametrize("degree", [3, 4])
def test_general_closed_form_c_zero(dtype, tol, degree):
    """C = 0: Z_n = Z_0^(d^n), so the count is the cap when |Z_0| <= 1 and
    otherwise the first n with |Z_0|^(2 d^n) > 4."""
    W = H = 48
    win = (-1.9, 1.9, -1.9, 1.9)
    cap = 30
    a = oracle.render(0j, win, W, H, cap, dtype, "julia", degree)
    checked = 0
    for j in range(H):
        for i in range(W):
            x, y = oracle.pixel_center(win, W, H, i, j)
            r = abs(complex(x, y))
            if abs(r - 1.0) < 1e-2:
                continue
            if r <= 1.0:
                want = cap
            else:
                L = math.log2(r)
                n = 0
                while (degree ** n) * L <= 1.0:  # |Z_n| = r^(d^n) <= 2
                    n += 1
                if any(abs(degree ** k * L - 1.0) < degree ** k * tol for k in (n - 1, n) if k >= 0):
                    continue
                want = min(n, cap)
            assert a[j, i] == want, (dtype, degree, i, j, r, a[j, i], want)
            checked += 1
    assert checked > 0.9 * W * H


@pytest.mark.parametrize("dtype", DTYPES)
def test_general_symmetries(dtype):
    """Conjugating C mirrors the image top to bottom (every operation is
    sign-symmetric); for even d, (-Z)^d = Z^d bit for bit, so the centred
    image is its own 180-degree rotation."""
    W, H, cap = 60, 44, 80
    win = (-1.4, 1.4, -1.1, 1.1)
    c = complex(-0.35, 0.52)
    for d in (3, 5):
        a = oracle.render(c, win, W, H, cap, dtype, "julia", d)
        b = oracle.render(c.conjugate(), win, W, H, cap, dtype, "julia", d)
        np.testing.assert_array_equal(b, a[::-1, :])
    for d in (4, 6):
        a = oracle.render(c, win, W, H, cap, dtype, "julia", d)
        np.testing.assert_array_equal(a, a[::-1, ::-1])


def test_general_exact_rational_counts_small_cap():
    """Brute force in exact rationals: Z^3 + C on an 8 x 8 grid with cap 5.
    The FP64 count must agree wherever no exact |Z_n|^2 lies within 1e-9 of 4."""
    win = (-1.3, 1.3, -1.3, 1.3)
    cr, ci = Fraction(-1, 5), Fraction(3, 10)
    cap, d = 5, 3
    got = oracle.render(complex(float(cr), float(ci)), win, 8, 8, cap, "fp64", "julia", d)
    compared = 0
    for j in range(8):
        for i in range(8):
            x0, y0 = oracle.pixel_center(win, 8, 8, i, j)
            x, y = Fraction(x0), Fraction(y0)
            n, close = 0, False
            while n < cap:
                m = x * x + y * y
                if abs(m - 4) < Fraction(1, 10 ** 9):
                    close = True
                if m > 4:
                    break
                wr, wi = x, y
                for _ in range(d - 1):
                    wr, wi = wr * x - wi * y, wr * y + wi * x
                x, y = wr + cr, wi + ci
                n += 1
            if not close:
                assert got[j, i] == n, (i, j, got[j, i], n)
                compared += 1
    assert compared >= 60


# ------------------------------------------- per-pixel entry points
# jro_render_pixels and jro_render_pixels_general check every sampled and
# full-size GPU test, and time the CPU baseline.  They must give, at any list
# of (column, row) pairs, the counts that the independent numpy
# implementation gives at those pixels of the whole image (and that the
# oracle's own whole-image loop gives).  The grid is not square and the list
# holds every pixel in a shuffled order, repeats and the four corners, so a
# swapped column/row, a swapped width/height, a shifted list index or a lost
# mode fails here.
PIXEL_CASES = [
    # c, window, W, H, cap, mode
    (complex(0.285, 0.01), (-1.3, 1.1, -0.7, 0.95), 29, 23, 80, "julia"),
    (0j, (-2.0, 0.7, -1.1, 1.2), 31, 19, 60, "mandelbrot"),
]


def _pixel_list(W, H, seed):
    rng = np.random.default_rng(seed)
    k = rng.permutation(W * H)
    ii, jj = (k % W), (k // W)
    extra = rng.integers(0, W * H, 40)
    ii = np.concatenate([ii, extra % W, [0, W - 1, 0, W - 1]])
    jj = np.concatenate([jj, extra // W, [0, 0, H - 1, H - 1]])
    return ii.astype(np.int32), jj.astype(np.int32)


@pytest.mark.parametrize("degree", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("case", range(len(PIXEL_CASES)))
@pytest.mark.parametrize("dtype", DTYPES)
def test_render_pixels_matches_whole_images(dtype, case, degree):
    c, win, W, H, cap, mode = PIXEL_CASES[case]
    ii, jj = _pixel_list(W, H, 7 * case + degree)
    got = oracle.render_pixels(c, win, W, H, cap, ii, jj, dtype, mode, degree)
    if degree == 2:
        twin = ind.render(c, win, W, H, cap, dtype, mode)
    else:
        twin = ind.render_general(c, win, W, H, cap, dtype, mode, degree)
    np.testing.assert_array_equal(got, twin[jj, ii])
    whole = oracle.render(c, win, W, H, cap, dtype, mode, degree)
    np.testing.assert_array_equal(got, whole[jj, ii])
    # the images must not be trivial: several distinct counts, some capped
    assert len(np.unique(got)) >= 5 and (got == cap).any()


# ------------------------- rational maps Z^d + C + lam / Z^d (two parameters)
# Orbits whose every value is dyadic: exact in binary64 and binary32, so the
# counts are those of exact arithmetic.  Each is worked by hand.
RATIONAL_ORBITS = [
    # degree, Z_0, C, lam, count (cap 100)
    (2, 1, 0, 1, 2),               # 1; 1 + 1/1 = 2 (|2|^2 = 4 is not > 4); 4 + 1/4
    (2, 1j, 0, -1, 2),             # i; -1 + (-1)/(-1) = 0; then 0/0: not a number
    (2, 0, 0, 1, 1),               # the pole itself: 0, then 0/0
    (2, 1, -1 - 1j, 1 + 1j, 100),  # lam / 1 cancels C: 1 is a fixed point
    (2, 1, 0, 1j, 2),              # 1; 1 + i; W = 2i, i/(2i) = 1/2: 1/2 + 2i
    (2, 1, 0, 1 + 1j, 1),          # 1; 2 + i
    (3, 1, 0, 2, 1),               # 1; 1 + 2 = 3
    (2, 3, 0, 1, 0),
    (2, 2, 0, 0, 1),               # lam = 0: 2; 4
    (2, 1, -1, 1, 100),            # 1 - 1 + 1 = 1
    (4, -1, -1, 1, 100),           # (-1)^4 = 1: 1 - 1 + 1 = 1, then 1 again
]
RATIONAL_DTYPES = ["fp64", "fp32"]


@pytest.mark.parametrize("dtype", RATIONAL_DTYPES)
def test_rational_exact_small_orbits(dtype):
    for d, z0, c, lam, want in RATIONAL_ORBITS:
        assert oracle.count(z0, c, 100, dtype, degree=d, lam=lam) == want, (d, z0, c, lam)
        assert oracle.count(z0, c, 1, dtype, degree=d, lam=lam) == min(want, 1)
        assert oracle.count(z0, c, 0, dtype, degree=d, lam=lam) == 0


@pytest.mark.parametrize("dtype", RATIONAL_DTYPES)
@pytest.mark.parametrize("degree", [2, 3, 5])
def test_rational_lambda_zero_is_the_polynomial_map(dtype, degree):
    """lam = 0 adds 0 / |W|^2 = +0 to each coordinate, which changes no
    nonzero value: the counts are those of Z^d + C (no iterate of these
    grids is exactly 0)."""
    for c, win in ((complex(0.4, 0.3), (-1.3, 1.3, -1.2, 1.2)),
                   (complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5))):
        a = oracle.render(c, win, 41, 30, 90, dtype, "julia", degree, lam=0j)
        b = oracle.render_general(c, win, 41, 30, 90, dtype, "julia", degree)
        np.testing.assert_array_equal(a, b)


RATIONAL_CASES = [
    # c, lam, window: each image holds escapes, bounded orbits and many
    # counts at degrees 2, 3 and 4 (an attracting cycle away from the pole)
    (complex(-0.55, 0.1), complex(-0.02, 0.01), (-1.5, 1.5, -1.2, 1.2)),
    (complex(-0.1, 0.65), complex(0.005, 0.005), (-1.3, 1.1, -0.9, 1.0)),
]


@pytest.mark.parametrize("dtype", RATIONAL_DTYPES)
@pytest.mark.parametrize("degree", [2, 3, 4])
def test_rational_matches_numpy_reimplementation(dtype, degree):
    for c, lam, win in RATIONAL_CASES:
        a = oracle.render(c, win, 37, 29, 70, dtype, "julia", degree, lam=lam)
        b = ind.render_rational(c, lam, win, 37, 29, 70, dtype, degree)
        np.testing.assert_array_equal(a, b)
        # the images are not trivial: escapes, interior and several counts
        assert len(np.unique(a)) >= 5 and (a == 70).any() and (a < 3).any()


@pytest.mark.parametrize("dtype", RATIONAL_DTYPES)
def test_rational_symmetries(dtype):
    """Conjugating C and lam mirrors the image top to bottom (every
    operation, the division included, is sign-symmetric); for even d the map
    is even, f(-Z) = f(Z) bit for bit, so the centred image is its own
    180-degree rotation."""
    W, H, cap = 60, 44, 80
    win = (-1.4, 1.4, -1.1, 1.1)
    c, lam = complex(-0.35, 0.52), complex(0.04, 0.03)
    for d in (2, 3, 4):
        a = oracle.render(c, win, W, H, cap, dtype, "julia", d, lam=lam)
        b = oracle.render(c.conjugate(), win, W, H, cap, dtype, "julia", d,
                          lam=lam.conjugate())
        np.testing.assert_array_equal(b, a[::-1, :])
        if d % 2 == 0:
            np.testing.assert_array_equal(a, a[::-1, ::-1])


@pytest.mark.parametrize("degree", [2, 3])
def test_rational_exact_rational_counts_small_cap(degree):
    """Brute force in exact rationals on an 8 x 8 grid with cap 4 (the exact
    values' sizes multiply by about 2d + 2 per step): the FP64 count must
    agree wherever no exact |Z_n|^2 lies within 1e-9 of 4."""
    win = (-1.3, 1.3, -1.3, 1.3)
    c, lam = complex(-0.25, 0.375), complex(0.0625, -0.03125)
    cr, ci, lr, li = (Fraction(v) for v in (c.real, c.imag, lam.real, lam.imag))
    cap = 4
    got = oracle.render(c, win, 8, 8, cap, "fp64", "julia", degree, lam=lam)
    compared = 0
    for j in range(8):
        for i in range(8):
            x0, y0 = oracle.pixel_center(win, 8, 8, i, j)
            x, y = Fraction(x0), Fraction(y0)
            n, close = 0, False
            while n < cap:
                m = x * x + y * y
                if abs(m - 4) < Fraction(1, 10 ** 9):
                    close = True
                if m > 4:
                    break
                wr, wi = x, y
                for _ in range(degree - 1):
                    wr, wi = wr * x - wi * y, wr * y + wi * x
                q = wr * wr + wi * wi          # nonzero: no grid orbit hits 0
                x, y = wr + cr + (lr * wr + li * wi) / q, wi + ci + (li * wr - lr * wi) / q
                n += 1
            if not close:
                assert got[j, i] == n, (i, j, got[j, i], n)
                compared += 1
    assert compared >= 56


@pytest.mark.parametrize("dtype", RATIONAL_DTYPES)
def test_render_pixels_rational_matches_whole_images(dtype):
    c, lam, win = RATIONAL_CASES[1]
    W, H, cap, d = 29, 23, 70, 3
    ii, jj = _pixel_list(W, H, 31)
    got = oracle.render_pixels(c, win, W, H, cap, ii, jj, dtype, "julia", d, lam=lam)
    np.testing.assert_array_equal(got, ind.render_rational(c, lam, win, W, H, cap, dtype,
                                                           d)[jj, ii])
    whole = oracle.render(c, win, W, H, cap, dtype, "julia", d, lam=lam)
    np.testing.assert_array_equal(got, whole[jj, ii])
    assert len(np.unique(got)) >= 5 and (got == cap).any()


# -------------------------------- prescribed cardioid path (Section 3)
def test_cardioid_constants_exact_quarter_turns():
    """step = i: u_k = i^k exactly, and with a = 4 every constant is dyadic:
    C = (2u - u^2) / 4 gives 1/4, 1/4 + i/2, -3/4, 1/4 - i/2, ... (k = 6
    tells the order of the square-and-multiply bits apart)."""
    want = [0.25 + 0j, 0.25 + 0.5j, -0.75 + 0j, 0.25 - 0.5j]
    for k in range(12):
        assert oracle.cardioid_constant(1j, 4.0, 0.0, k) == want[k % 4], k
    # a_k = a0 - da k: a_1 = 3.5, C_1 = (1 + 2i) / 3.5 correctly rounded
    assert oracle.cardioid_constant(1j, 4.0, 0.5, 1) == complex(
        float(Fraction(1) / Fraction(7, 2)), float(Fraction(2) / Fraction(7, 2)))
    assert oracle.cardioid_constant(1j, 4.0, 0.25, 6) == -3.0 / 2.5 + 0j   # u = -1, a = 2.5


def test_cardioid_constants_against_high_precision():
    """The exact power of the binary64 step, in 60-digit arithmetic, and the
    definition's own rounded a_k: every constant within 1e-13 relative for
    k < 4096 (u_k takes up to 2 log2(k) + 1 rounded complex products).  And within 1e-13 of the closed form with t_k = 2 pi k / n for
    the first trips."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    n, a0, da = 64, 3.9, 0.4 / 255
    step = complex(math.cos(2 * math.pi / n), math.sin(2 * math.pi / n))
    s = mpmath.mpc(step.real, step.imag)
    for k in list(range(0, 300)) + [511, 1000, 2047, 4095]:
        got = oracle.cardioid_constant(step, a0, da, k)
        u = s ** k
        ak = a0 - da * k                     # binary64, as the definition rounds it
        want = (2 * u - u * u) / ak
        err = abs(mpmath.mpc(got.real, got.imag) - want) / abs(want)
        assert err < 1e-13, (k, float(err))
        if k < 256:
            t = 2 * math.pi * k / n
            closed = complex((2 * math.cos(t) - math.cos(2 * t)) / ak,
                             (2 * math.sin(t) - math.sin(2 * t)) / ak)
            assert abs(got - closed) < 1e-13, k


def test_cardioid_a4_is_the_main_cardioid():
    """With a = 4, C = u/2 - u^2/4, so 1 - 4C = (1 - u)^2 and the fixed point
    (1 - sqrt(1 - 4C)) / 2 has multiplier u: modulus 1, the border of the
    main cardioid of the Mandelbrot set (Section 3)."""
    step = complex(math.cos(2 * math.pi / 64), math.sin(2 * math.pi / 64))
    for k in range(1, 64):
        c = oracle.cardioid_constant(step, 4.0, 0.0, k)
        mult = 1 - np.sqrt(1 - 4 * c)
        assert abs(abs(mult) - 1.0) < 1e-13, k


def test_cardioid_path_passes_the_paper_constants():
    """The four constants of Figure 2 lie on the a = 3.9 cardioid: the path
    with 2^16 frames per trip passes within 5e-5 of each."""
    rows = {r[0]: complex(float(r[1]), float(r[2])) for r in read_table("paper_constants.txt")}
    consts = [rows[k] for k in ("fig2_a", "fig2_b", "fig2_c", "fig2_d")]
    n = 1 << 16
    step = complex(math.cos(2 * math.pi / n), math.sin(2 * math.pi / n))
    pts = np.array([oracle.cardioid_constant(step, 3.9, 0.0, k) for k in range(0, n, 1)])
    for c in consts:
        assert np.abs(pts - c).min() < 5e-5, c
