"""ctypes wrapper of the CPU oracle (oracle/julia_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain single-threaded CPU implementation of the
escape-time counts that the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import it;
the product package never does, and this module imports nothing from it.

Method: Mayfield et al., Section 2 (escape-time iteration Z_{n+1} = Z_n^2 + C
over pixels scaled onto the complex plane, capped at max_iter) and Section 3
(Mandelbrot variant, C from the pixel, Z_0 = 0).  The readings of the paper the
oracle takes are listed in ``julia_oracle.h``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DTYPES = {"fp64": 0, "fp32": 1, "ff": 2}
MODES = {"julia": 0, "mandelbrot": 1}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "julia_oracle.c")
    if (not os.path.exists(_LIB_PATH)
            or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src)):
        from . import build_oracle
        build_oracle.build()
    _lib = _open(_LIB_PATH)
    return _lib


def _open(path):
    """Load an oracle build and declare its C signatures."""
    lib = ctypes.CDLL(path)
    d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    p_i32 = ctypes.POINTER(ctypes.c_int32)
    p_f = ctypes.POINTER(ctypes.c_float)
    p_d = ctypes.POINTER(ctypes.c_double)
    f = ctypes.c_float
    lib.jro_render.argtypes = [i32, i32, d, d, d, d, d, d, i32, i32, i32, p_i32]
    lib.jro_render.restype = None
    lib.jro_render_pixels.argtypes = [i32, i32, d, d, d, d, d, d, i32, i32, i32,
                                      i64, p_i32, p_i32, p_i32]
    lib.jro_render_pixels.restype = None
    lib.jro_pixel_center.argtypes = [d, d, d, d, i32, i32, i32, i32, p_d, p_d]
    lib.jro_pixel_center.restype = None
    lib.jro_count.argtypes = [i32, d, d, d, d, i32]
    lib.jro_count.restype = i32
    for name in ("jro_two_sum", "jro_fast_two_sum", "jro_two_prod"):
        getattr(lib, name).argtypes = [f, f, p_f, p_f]
        getattr(lib, name).restype = None
    for name in ("jro_dw_add", "jro_dw_mul", "jro_dw_add_cheap"):
        getattr(lib, name).argtypes = [f, f, f, f, p_f, p_f]
        getattr(lib, name).restype = None
    lib.jro_dw_sqr.argtypes = [f, f, p_f, p_f]
    lib.jro_dw_sqr.restype = None
    lib.jro_dw_split.argtypes = [d, p_f, p_f]
    lib.jro_dw_split.restype = None
    lib.jro_count_general.argtypes = [i32, i32, d, d, d, d, i32]
    lib.jro_count_general.restype = i32
    lib.jro_render_general.argtypes = [i32, i32, i32, d, d, d, d, d, d, i32, i32, i32, p_i32]
    lib.jro_render_general.restype = None
    lib.jro_render_pixels_general.argtypes = [i32, i32, i32, d, d, d, d, d, d, i32, i32, i32,
                                              i64, p_i32, p_i32, p_i32]
    lib.jro_render_pixels_general.restype = None
    lib.jro_count_rational.argtypes = [i32, i32, d, d, d, d, d, d, i32]
    lib.jro_count_rational.restype = i32
    lib.jro_render_rational.argtypes = [i32, i32, d, d, d, d, d, d, d, d, i32, i32, i32, p_i32]
    lib.jro_render_rational.restype = None
    lib.jro_render_pixels_rational.argtypes = [i32, i32, d, d, d, d, d, d, d, d, i32, i32, i32,
                                               i64, p_i32, p_i32, p_i32]
    lib.jro_render_pixels_rational.restype = None
    lib.jro_cardioid_constant.argtypes = [d, d, d, d, i32, p_d, p_d]
    lib.jro_cardioid_constant.restype = None
    p_u32 = ctypes.POINTER(ctypes.c_uint32)
    lib.jro_colorize.argtypes = [p_i32, i64, p_u32, i32, p_u32]
    lib.jro_colorize.restype = None
    return lib


def _as_ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _rational_args(dtype, mode, lam):
    if mode != "julia" or dtype not in ("fp64", "fp32"):
        raise ValueError("the rational maps have Julia images in fp64 and fp32 only")
    lam = complex(lam)
    return lam.real, lam.imag


def render(c, window, width, height, max_iter, dtype="fp64", mode="julia", degree=2,
           lam=None):
    """Counts of a whole image: int32 array of shape (height, width), row 0 = im_max.

    ``c`` is a complex (ignored in Mandelbrot mode); ``window`` is
    (re_min, re_max, im_min, im_max).  ``degree`` 3..8 iterates the general
    map Z^d + C (jro_render_general); 2 is the paper's Z^2 + C.  With ``lam``
    (a complex) the map is the rational Z^d + C + lam / Z^d
    (jro_render_rational; Julia images, fp64 or fp32).
    """
    lib = _load()
    c = complex(c)
    out = np.empty((int(height), int(width)), dtype=np.int32)
    if lam is not None:
        lr, li = _rational_args(dtype, mode, lam)
        lib.jro_render_rational(DTYPES[dtype], int(degree), c.real, c.imag, lr, li,
                                *[float(v) for v in window], int(width), int(height),
                                int(max_iter), _as_ptr(out))
    elif degree == 2:
        lib.jro_render(DTYPES[dtype], MODES[mode], c.real, c.imag,
                       *[float(v) for v in window], int(width), int(height),
                       int(max_iter), _as_ptr(out))
    else:
        lib.jro_render_general(DTYPES[dtype], MODES[mode], int(degree), c.real, c.imag,
                               *[float(v) for v in window], int(width), int(height),
                               int(max_iter), _as_ptr(out))
    return out


def render_general(c, window, width, height, max_iter, dtype="fp64", mode="julia", degree=2):
    """The general-map formulation for any degree 2..8, d = 2 included."""
    lib = _load()
    c = complex(c)
    out = np.empty((int(height), int(width)), dtype=np.int32)
    lib.jro_render_general(DTYPES[dtype], MODES[mode], int(degree), c.real, c.imag,
                           *[float(v) for v in window], int(width), int(height),
                           int(max_iter), _as_ptr(out))
    return out


def render_pixels(c, window, width, height, max_iter, ii, jj, dtype="fp64",
                  mode="julia", degree=2, lam=None):
    """Counts at the pixels (column ii[k], row jj[k]) of the image ``render`` gives."""
    lib = _load()
    c = complex(c)
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    assert ii.shape == jj.shape and ii.ndim == 1
    out = np.empty(ii.shape, dtype=np.int32)
    if lam is not None:
        lr, li = _rational_args(dtype, mode, lam)
        lib.jro_render_pixels_rational(DTYPES[dtype], int(degree), c.real, c.imag, lr, li,
                                       *[float(v) for v in window], int(width), int(height),
                                       int(max_iter), ii.size, _as_ptr(ii), _as_ptr(jj),
                                       _as_ptr(out))
    elif degree == 2:
        lib.jro_render_pixels(DTYPES[dtype], MODES[mode], c.real, c.imag,
                              *[float(v) for v in window], int(width), int(height),
                              int(max_iter), ii.size, _as_ptr(ii), _as_ptr(jj),
                              _as_ptr(out))
    else:
        lib.jro_render_pixels_general(DTYPES[dtype], MODES[mode], int(degree), c.real, c.imag,
                                      *[float(v) for v in window], int(width), int(height),
                                      int(max_iter), ii.size, _as_ptr(ii), _as_ptr(jj),
                                      _as_ptr(out))
    return out


def colorize(counts, palette):
    """Colour levels of a count image: out[k] = palette[min(counts[k], len - 1)]
    as a uint32 array of the counts' shape (Section 2: a pixel's colour level
    follows from its iteration count)."""
    lib = _load()
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    palette = np.ascontiguousarray(palette, dtype=np.uint32)
    assert palette.ndim == 1 and palette.size >= 1 and (counts >= 0).all()
    out = np.empty(counts.shape, dtype=np.uint32)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    lib.jro_colorize(_as_ptr(counts), counts.size, palette.ctypes.data_as(u32), palette.size,
                     out.ctypes.data_as(u32))
    return out


def pixel_center(window, width, height, i, j):
    lib = _load()
    x, y = ctypes.c_double(), ctypes.c_double()
    lib.jro_pixel_center(*[float(v) for v in window], int(width), int(height),
                         int(i), int(j), ctypes.byref(x), ctypes.byref(y))
    return x.value, y.value


def count(z0, c, max_iter, dtype="fp64", degree=None, lam=None):
    """Count of one orbit with explicit Z_0 and C.  ``degree`` None: the
    Z^2 + C formulations; 2..8: the general-map formulations; with ``lam``
    the rational map Z^d + C + lam / Z^d (degree None means 2)."""
    lib = _load()
    z0, c = complex(z0), complex(c)
    if lam is not None:
        lr, li = _rational_args(dtype, "julia", lam)
        return int(lib.jro_count_rational(DTYPES[dtype], int(degree or 2), z0.real, z0.imag,
                                          c.real, c.imag, lr, li, int(max_iter)))
    if degree is None:
        return int(lib.jro_count(DTYPES[dtype], z0.real, z0.imag, c.real, c.imag,
                                 int(max_iter)))
    return int(lib.jro_count_general(DTYPES[dtype], int(degree), z0.real, z0.imag, c.real,
                                     c.imag, int(max_iter)))


def _pair(fn, *args):
    lib = _load()
    a, b = ctypes.c_float(), ctypes.c_float()
    getattr(lib, fn)(*args, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def two_sum(a, b):
    return _pair("jro_two_sum", a, b)


def fast_two_sum(a, b):
    return _pair("jro_fast_two_sum", a, b)


def two_prod(a, b):
    return _pair("jro_two_prod", a, b)


def dw_add(x, y):
    return _pair("jro_dw_add", x[0], x[1], y[0], y[1])


def dw_mul(x, y):
    return _pair("jro_dw_mul", x[0], x[1], y[0], y[1])


def dw_sqr(x):
    return _pair("jro_dw_sqr", x[0], x[1])


def dw_add_cheap(x, y):
    return _pair("jro_dw_add_cheap", x[0], x[1], y[0], y[1])


def dw_split(v):
    return _pair("jro_dw_split", float(v))


def cardioid_constant(step, a0, da, k):
    """The constant of frame k of a prescribed cardioid path (Section 3):
    (2 u_k - u_k^2) / (a0 - da k) with u_k = step^k by square-and-multiply
    (jro_cardioid_constant)."""
    lib = _load()
    step = complex(step)
    cr, ci = ctypes.c_double(), ctypes.c_double()
    lib.jro_cardioid_constant(step.real, step.imag, float(a0), float(da), int(k),
                              ctypes.byref(cr), ctypes.byref(ci))
    return complex(cr.value, ci.value)
