"""Seeded synthetic inputs for the escape-time workloads.

This module is shared by the GPU library's tests and benchmark and by the
oracle's tests.  It holds the parameter recipes only -- complex constants,
windows, image sizes, iteration caps, arrival times -- and none of the per-pixel
arithmetic; both sides receive the same binary64 parameters from here.

The one piece of orbit arithmetic here is the acceptance rule of the uneven
batch's constant sampler (``accept_c``): a candidate C is kept when its
Mandelbrot orbit from 0 stays within |Z|^2 <= 4 for 20 steps.  It only decides
which constants make up the workload; no count is ever compared against it.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014; the constants are those of the
published generator), mapped to [0, 1) as (x >> 11) * 2^-53.

The paper (Mayfield et al.) evaluates on no dataset: its inputs are a constant
C, a window and an image size (Section 2; square images from 10x10 to
10000x10000 pixels in its timing study; iteration cap 100).  The recipes below
follow that shape.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (64-bit state, Weyl increment 0x9E3779B97F4A7C15)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """U[0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))

    def exponential(self, rate: float) -> float:
        return -math.log(1.0 - self.uniform()) / rate


@dataclass
class Frame:
    """One image request: constant, window, size, cap, arithmetic, variant."""
    c: complex
    window: Tuple[float, float, float, float]  # re_min, re_max, im_min, im_max
    width: int
    height: int
    max_iter: int
    dtype: str = "fp64"        # "fp64" | "fp32" | "ff"
    mode: str = "julia"        # "julia" | "mandelbrot"
    degree: int = 2            # map Z^degree + C
    lam: Optional[complex] = None  # set: the rational map Z^degree + C + lam / Z^degree

    @property
    def pixels(self) -> int:
        return self.width * self.height


# --------------------------------------------------------------------------
# Single image, 512x512, C = -0.8 + 0.156i, window [-1.5, 1.5]^2, cap 100.
# --------------------------------------------------------------------------
def single_512(dtype: str = "fp64") -> Frame:
    return Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 512, 512, 100, dtype)


# --------------------------------------------------------------------------
# Single image 4096x4096, window [-1.6, 1.6]^2, C = 0.7885 exp(i theta),
# theta = 2 pi u from the seed; cap 100 or 1000.
# --------------------------------------------------------------------------
def single_4096(seed: int, max_iter: int, dtype: str, side: int = 4096) -> Frame:
    theta = 2.0 * math.pi * SplitMix64(seed).uniform()
    c = complex(0.7885 * math.cos(theta), 0.7885 * math.sin(theta))
    return Frame(c, (-1.6, 1.6, -1.6, 1.6), side, side, max_iter, dtype)


# --------------------------------------------------------------------------
# Parameter path: n frames of 1920x1080, C_k = 0.7885 exp(2 pi i k / n),
# window Re[-1.78, 1.78] x Im[-1, 1], cap 100, FP32.
# --------------------------------------------------------------------------
def parameter_path(n: int = 256, width: int = 1920, height: int = 1080,
                   max_iter: int = 100, dtype: str = "fp32") -> List[Frame]:
    frames = []
    for k in range(n):
        t = 2.0 * math.pi * k / n
        c = complex(0.7885 * math.cos(t), 0.7885 * math.sin(t))
        frames.append(Frame(c, (-1.78, 1.78, -1.0, 1.0), width, height, max_iter, dtype))
    return frames


# --------------------------------------------------------------------------
# Cardioid path of Section 3: f(t) = ((2 cos t - cos 2t)/a, (2 sin t - sin 2t)/a),
# a = 3.9 just outside the main cardioid (a = 4 is its border).
# --------------------------------------------------------------------------
def cardioid_point(t: float, a: float = 3.9) -> complex:
    return complex((2.0 * math.cos(t) - math.cos(2.0 * t)) / a,
                   (2.0 * math.sin(t) - math.sin(2.0 * t)) / a)


@dataclass
class GrowingCardioid:
    """Parameters of a prescribed cardioid path with a growing cardioid: the
    per-frame rotation step = e^{2 pi i / per_trip} (formed here once, with
    libm), a_k = a0 - da k from a0 down to a1 over the frames.  Each side
    (the device generator, the oracle) forms C_k from these itself."""
    step: complex
    a0: float
    da: float
    window: Tuple[float, float, float, float]
    frames: int
    width: int
    height: int
    max_iter: int
    dtype: str


def growing_cardioid_path(frames: int = 256, per_trip: int = 64, a0: float = 3.9,
                          a1: float = 3.5, width: int = 1920, height: int = 1080,
                          max_iter: int = 100, dtype: str = "fp32",
                          window=(-1.78, 1.78, -1.0, 1.0)) -> GrowingCardioid:
    """Section 3: the cardioid path with a = 3.9, then a growing cardioid
    (a decreasing) over several trips around the Mandelbrot set."""
    t = 2.0 * math.pi / per_trip
    da = (a0 - a1) / (frames - 1) if frames > 1 else 0.0
    return GrowingCardioid(complex(math.cos(t), math.sin(t)), a0, da, window, frames, width,
                           height, max_iter, dtype)


def cardioid_path(n: int, a: float = 3.9, width: int = 1920, height: int = 1080,
                  max_iter: int = 100, dtype: str = "fp32",
                  window=(-1.78, 1.78, -1.0, 1.0)) -> List[Frame]:
    return [Frame(cardioid_point(2.0 * math.pi * k / n, a), window, width, height,
                  max_iter, dtype) for k in range(n)]


# --------------------------------------------------------------------------
# General maps: a path of constants C_k = r exp(2 pi i k / n) for Z^d + C
# (r = 0.6 for d = 3 runs from light frames, mean count about 3, to frames
# with a mean near 45 at cap 100).
# --------------------------------------------------------------------------
def general_path(n: int = 32, degree: int = 3, radius: float = 0.6, width: int = 1920,
                 height: int = 1080, max_iter: int = 100, dtype: str = "fp32",
                 window=(-1.6, 1.6, -0.9, 0.9)) -> List[Frame]:
    return [Frame(complex(radius * math.cos(2.0 * math.pi * k / n),
                          radius * math.sin(2.0 * math.pi * k / n)),
                  window, width, height, max_iter, dtype, "julia", degree) for k in range(n)]


# --------------------------------------------------------------------------
# Mandelbrot zoom (Section 3's minimap and deep zooms on M): n frames of the
# Mandelbrot image, the window's width shrinking geometrically from w0 to w1
# around a boundary point in the seahorse valley; cap 1000, FP64.
# --------------------------------------------------------------------------
ZOOM_CENTRE = complex(-0.743643887037151, 0.131825904205330)


def mandelbrot_zoom(n: int = 64, w0: float = 3.0, w1: float = 1e-5, width: int = 1920,
                    height: int = 1080, max_iter: int = 1000, dtype: str = "fp64",
                    centre: complex = ZOOM_CENTRE) -> List[Frame]:
    out = []
    for k in range(n):
        w = w0 * (w1 / w0) ** (k / (n - 1) if n > 1 else 0.0)
        h = w * height / width
        win = (centre.real - w / 2, centre.real + w / 2, centre.imag - h / 2, centre.imag + h / 2)
        out.append(Frame(0j, win, width, height, max_iter, dtype, "mandelbrot"))
    return out


# --------------------------------------------------------------------------
# Rational path: n frames of Z^d + C_k + lam_k / Z^d, C_k on the parameter
# path's circle (|C| = 0.7885) and lam_k = lam_radius exp(-2 pi i k / n)
# turning the other way; the parameter path's window.  |C| + |lam| / 2^d <= 1.9,
# so escape is absorbing in every frame.
# --------------------------------------------------------------------------
def rational_path(n: int = 32, degree: int = 2, lam_radius: float = 0.002, width: int = 1920,
                  height: int = 1080, max_iter: int = 100, dtype: str = "fp32",
                  window=(-1.78, 1.78, -1.0, 1.0)) -> List[Frame]:
    out = []
    for k in range(n):
        t = 2.0 * math.pi * k / n
        c = complex(0.7885 * math.cos(t), 0.7885 * math.sin(t))
        lam = complex(lam_radius * math.cos(-t), lam_radius * math.sin(-t))
        out.append(Frame(c, window, width, height, max_iter, dtype, "julia", degree, lam))
    return out


# --------------------------------------------------------------------------
# Uneven batch: square side ~ U{256..4096}; C uniform on the unit disk,
# accepted when its Mandelbrot orbit from 0 survives 20 steps; cap from
# {100, 500, 2000}; FP32 or float-float with probability 1/2 each.
# --------------------------------------------------------------------------
ACCEPT_STEPS = 20


def accept_c(c: complex, steps: int = ACCEPT_STEPS) -> bool:
    """True when |Z_n|^2 <= 4 for n = 0..steps-1 on the orbit Z_0 = 0, Z' = Z^2 + c."""
    x = y = 0.0
    for _ in range(steps):
        if x * x + y * y > 4.0:
            return False
        x, y = x * x - y * y + c.real, 2.0 * x * y + c.imag
    return True


def sample_c_disk(rng: SplitMix64) -> complex:
    while True:
        u = 2.0 * rng.uniform() - 1.0
        v = 2.0 * rng.uniform() - 1.0
        if u * u + v * v > 1.0:
            continue
        c = complex(u, v)
        if accept_c(c):
            return c


def uneven_batch(seed: int = 0, n: int = 1024, side_lo: int = 256, side_hi: int = 4096,
                 caps=(100, 500, 2000), dtypes=("fp32", "ff")) -> List[Frame]:
    rng = SplitMix64(seed)
    frames = []
    for _ in range(n):
        side = rng.randint(side_lo, side_hi)
        c = sample_c_disk(rng)
        cap = caps[rng.randint(0, len(caps) - 1)]
        dt = dtypes[rng.randint(0, len(dtypes) - 1)]
        frames.append(Frame(c, (-1.6, 1.6, -1.6, 1.6), side, side, cap, dt))
    return frames


# --------------------------------------------------------------------------
# Serving: Poisson arrivals; each request a random C (uneven-batch sampler),
# window centre U[-1.5, 1.5]^2, width log-uniform in [1e-9, 3], size from
# {640x480, 1280x720, 1920x1080}, cap U{100..5000}.  The arithmetic is left to
# the precision policy of the serving loop (dtype "auto" here).
# --------------------------------------------------------------------------
SERVE_SIZES = ((640, 480), (1280, 720), (1920, 1080))


@dataclass
class Request:
    arrival_s: float
    frame: Frame
    rid: int = 0


def serving_stream(seed: int, rate_per_s: float, n: int,
                   width_lo: float = 1e-9, width_hi: float = 3.0,
                   cap_lo: int = 100, cap_hi: int = 5000,
                   sizes=SERVE_SIZES) -> List[Request]:
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(rate_per_s)
        c = sample_c_disk(rng)
        cre = -1.5 + 3.0 * rng.uniform()
        cim = -1.5 + 3.0 * rng.uniform()
        width = math.exp(math.log(width_lo) + rng.uniform() * (math.log(width_hi) - math.log(width_lo)))
        w, h = sizes[rng.randint(0, len(sizes) - 1)]
        height = width * h / w
        cap = rng.randint(cap_lo, cap_hi)
        win = (cre - 0.5 * width, cre + 0.5 * width, cim - 0.5 * height, cim + 0.5 * height)
        out.append(Request(t, Frame(c, win, w, h, cap, "auto"), k))
    return out


# --------------------------------------------------------------------------
# Square-image sweep in the shape of the paper's timing study (Section 2,
# Figure 1): sides from 10 to 10000 pixels, cap 100.
# --------------------------------------------------------------------------
FIG1_SIDES = (10, 32, 100, 316, 1000, 3162, 10000)


def square_sweep(dtype: str = "fp64", sides=FIG1_SIDES) -> List[Frame]:
    base = single_512(dtype)
    return [Frame(base.c, base.window, s, s, 100, dtype) for s in sides]


# --------------------------------------------------------------------------
# Precision windows: the serving stream's windows at one fixed width.  Each
# window has a constant from the uneven-batch sampler and a centre uniform in
# [-1.5, 1.5]^2, is `width` wide with the 640x480 aspect, and is probed at
# `pixels` pixel positions drawn uniformly from its 640x480 grid.
# --------------------------------------------------------------------------
PRECISION_WIDTHS = (3.0, 1e-1, 1e-3, 1e-5, 1e-7, 1e-9)
PRECISION_CAPS = (100, 1000, 5000)


@dataclass
class ProbeWindow:
    frame: Frame          # 640 x 480, dtype left to the caller
    ii: List[int]         # probed columns
    jj: List[int]         # probed rows


def precision_windows(seed: int, width: float, max_iter: int, n: int = 32,
                      pixels: int = 1024, size=(640, 480)) -> List[ProbeWindow]:
    rng = SplitMix64(seed)
    W, H = size
    out = []
    for _ in range(n):
        c = sample_c_disk(rng)
        cre = -1.5 + 3.0 * rng.uniform()
        cim = -1.5 + 3.0 * rng.uniform()
        height = width * H / W
        win = (cre - 0.5 * width, cre + 0.5 * width, cim - 0.5 * height, cim + 0.5 * height)
        ii = [rng.randint(0, W - 1) for _ in range(pixels)]
        jj = [rng.randint(0, H - 1) for _ in range(pixels)]
        out.append(ProbeWindow(Frame(c, win, W, H, max_iter, "fp64"), ii, jj))
    return out


def precision_seed(width: float, max_iter: int, kind: str = "serving") -> int:
    """The seed of a (width, cap) cell of the precision table."""
    base = 1000 if kind == "serving" else 5000
    return base + 10 * PRECISION_WIDTHS.index(width) + PRECISION_CAPS.index(max_iter)


# --------------------------------------------------------------------------
# Windows centred on the Julia set itself: what an exploring user zooms into,
# and the hardest case for a short arithmetic (neighbouring pixels have very
# different counts).  The centre is found without any escape-time count, from
# two facts about the map f(z) = z^2 + c:
#   * its fixed point beta = (1 + sqrt(1 - 4c)) / 2 (principal root) has
#     multiplier |2 beta| = |1 + sqrt(1 - 4c)| >= 1 (the root's real part is
#     not negative), so it is repelling, or parabolic at c = 1/4, and such a
#     fixed point lies in the Julia set J(c);
#   * J(c) is completely invariant, so both preimages +-sqrt(z - c) of a point
#     of J(c) lie in J(c) (the inverse-iteration construction of J).
# `steps` preimages with random branches move the centre off beta along J.
# --------------------------------------------------------------------------
def julia_set_point(c: complex, rng: SplitMix64, steps: int = 12) -> complex:
    import cmath
    z = 0.5 * (1.0 + cmath.sqrt(1.0 - 4.0 * c))
    for _ in range(steps):
        z = cmath.sqrt(z - c)
        if rng.uniform() < 0.5:
            z = -z
    return z


def boundary_windows(seed: int, width: float, max_iter: int, n: int = 32,
                     pixels: int = 1024, size=(640, 480)) -> List[ProbeWindow]:
    """precision_windows with each window centred on a point of J(C)."""
    rng = SplitMix64(seed)
    W, H = size
    out = []
    for _ in range(n):
        c = sample_c_disk(rng)
        z = julia_set_point(c, rng)
        height = width * H / W
        win = (z.real - 0.5 * width, z.real + 0.5 * width,
               z.imag - 0.5 * height, z.imag + 0.5 * height)
        ii = [rng.randint(0, W - 1) for _ in range(pixels)]
        jj = [rng.randint(0, H - 1) for _ in range(pixels)]
        out.append(ProbeWindow(Frame(c, win, W, H, max_iter, "fp64"), ii, jj))
    return out


def probe_windows(kind: str, width: float, max_iter: int, **kw) -> List[ProbeWindow]:
    """The windows of one cell of the precision table: kind "serving" (the
    serving stream's centres) or "boundary" (centred on the Julia set)."""
    seed = precision_seed(width, max_iter, kind)
    if kind == "serving":
        return precision_windows(seed, width, max_iter, **kw)
    if kind == "boundary":
        return boundary_windows(seed, width, max_iter, **kw)
    raise ValueError(kind)
