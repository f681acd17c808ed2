"""Python binding of libjulia.so: escape-time Julia / Mandelbrot counts on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``csrc/``; torch supplies device memory and streams.  The library
must be built (``python paper_1611_03079_amd/build.py``); importing this module
without it raises, and nothing here falls back to a CPU path.

Method: Mayfield et al., Section 2 (iterate Z^2 + C from pixels scaled onto a
window, count iterations until |Z|^2 > 4, capped) and Section 3 (Mandelbrot
variant).  Conventions are those of ``include/julia.h``.
"""
import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjulia.so")

JR_OK, JR_EINVAL, JR_ENOMEM, JR_ENODEV, JR_ELAUNCH, JR_EINTERNAL = 0, -1, -2, -3, -4, -5
DTYPES = {"fp64": 0, "fp32": 1, "ff": 2}
MODES = {"julia": 0, "mandelbrot": 1}
ORDERS = {"table": 0, "cost": 1}
KERNELS = {"tiled": 0, "plain": 1, "hybrid": 2, "rows": 3}


class JuliaError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


class jr_complex(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class jr_window(ctypes.Structure):
    _fields_ = [("re_min", ctypes.c_double), ("re_max", ctypes.c_double),
                ("im_min", ctypes.c_double), ("im_max", ctypes.c_double)]


class jr_frame(ctypes.Structure):
    _fields_ = [("c", jr_complex), ("w", jr_window),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("row_begin", ctypes.c_int32),
                ("row_end", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("out_offset", ctypes.c_int64), ("map", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lam", jr_complex)]


class jr_schedule(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("defer", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("bail", ctypes.c_int32),
                ("handoff", ctypes.c_int32)]


assert ctypes.sizeof(jr_frame) == 112


class jr_cardioid_path(ctypes.Structure):
    _fields_ = [("step", jr_complex), ("a0", ctypes.c_double), ("da", ctypes.c_double),
                ("w", jr_window), ("frames", ctypes.c_int32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("out_offset", ctypes.c_int64)]


@dataclass(frozen=True)
class CardioidPath:
    """A prescribed cardioid path whose constants the device generates
    (julia_render_cardioid_path): frame k has C_k = (2 u_k - u_k^2) /
    (a0 - da k), u_k = step^k, rendered on `window` at width x height."""
    step: complex
    a0: float
    da: float
    window: tuple
    frames: int
    width: int
    height: int
    max_iter: int
    dtype: str = "fp32"

    def to_c(self, out_offset: int = 0) -> jr_cardioid_path:
        st = complex(self.step)
        return jr_cardioid_path(jr_complex(st.real, st.imag), float(self.a0), float(self.da),
                                _window(self.window), int(self.frames), int(self.width),
                                int(self.height), int(self.max_iter), DTYPES[self.dtype], 0,
                                int(out_offset))


@dataclass(frozen=True)
class Schedule:
    """Schedule of the tiled kernel (see include/julia.h); never changes counts."""
    tile_w: int = 64
    tile_h: int = 16
    unroll: int = 4
    defer: int = 0
    refill: int = 16
    persistent: int = 1
    waves_per_cu: int = 16
    order: str = "cost"
    kernel: str = "tiled"
    bail: int = 8
    handoff: int = 0

    def to_c(self) -> jr_schedule:
        return jr_schedule(self.tile_w, self.tile_h, self.unroll, self.defer, self.refill,
                           self.persistent, self.waves_per_cu, ORDERS[self.order],
                           KERNELS[self.kernel], self.bail, self.handoff)

    @staticmethod
    def from_c(s: jr_schedule) -> "Schedule":
        inv = {v: k for k, v in ORDERS.items()}
        invk = {v: k for k, v in KERNELS.items()}
        return Schedule(s.tile_w, s.tile_h, s.unroll, s.defer, s.refill, s.persistent,
                        s.waves_per_cu, inv[s.order], invk[s.kernel], s.bail, s.handoff)


EXPORTS = (
    "julia_render", "julia_render_plain", "mandelbrot_render", "mandelbrot_render_plain",
    "julia_render_batch", "julia_render_batch_noalloc", "julia_render_batch_colored",
    "julia_render_colored", "julia_render_cardioid_path", "jr_plan_create_cardioid",
    "jr_plan_create", "jr_plan_set_palette", "jr_plan_set_progress", "jr_set_image_schedule", "jr_get_image_schedule",
    "jr_clear_image_schedules", "jr_plan_launch", "jr_plan_capture",
    "jr_plan_replay", "jr_plan_info", "jr_plan_destroy", "jr_get_default_schedule",
    "jr_set_default_schedule", "jr_check_schedule", "jr_check_frames", "jr_strerror",
    "jr_last_error_message", "jr_device_info", "jr_shutdown",
)


def _load():
    # torch ships its own HIP runtime (libamdhip64.so.7 under torch/lib).  Loading
    # torch first makes libjulia.so bind to that same runtime (same SONAME), so
    # torch's device pointers and streams are valid in the library's calls and
    # the process holds one HIP runtime, not two.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libjulia.so is not built (%s); run python paper_1611_03079_amd/build.py"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = set()
    with open("/proc/self/maps") as maps:
        for line in maps:
            if "libamdhip64" in line:
                runtimes.add(line.split()[-1])
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); import torch before any other "
                          "HIP library" % ", ".join(sorted(runtimes)))
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER
    img = [jr_complex, jr_window, i32, i32, i32, i32, vp, vp]
    for name in ("julia_render", "julia_render_plain"):
        getattr(lib, name).argtypes = img
        getattr(lib, name).restype = ctypes.c_int
    for name in ("mandelbrot_render", "mandelbrot_render_plain"):
        getattr(lib, name).argtypes = img[1:]
        getattr(lib, name).restype = ctypes.c_int
    lib.julia_render_batch.argtypes = [P(jr_frame), i32, vp, i64, P(jr_schedule), vp]
    lib.julia_render_batch.restype = ctypes.c_int
    lib.julia_render_batch_noalloc.argtypes = [P(jr_frame), i32, vp, i64, P(jr_schedule), vp]
    lib.julia_render_batch_noalloc.restype = ctypes.c_int
    lib.julia_render_cardioid_path.argtypes = [P(jr_cardioid_path), vp, i64, P(jr_schedule), vp]
    lib.julia_render_cardioid_path.restype = ctypes.c_int
    lib.jr_plan_create_cardioid.argtypes = [P(jr_cardioid_path), vp, i64, P(jr_schedule), P(vp)]
    lib.jr_plan_create_cardioid.restype = ctypes.c_int
    lib.julia_render_batch_colored.argtypes = [P(jr_frame), i32, vp, i32, vp, i64,
                                               P(jr_schedule), vp]
    lib.julia_render_batch_colored.restype = ctypes.c_int
    lib.julia_render_colored.argtypes = [jr_complex, jr_window, i32, i32, i32, i32, vp, i32,
                                         vp, vp]
    lib.julia_render_colored.restype = ctypes.c_int
    lib.jr_plan_set_palette.argtypes = [vp, vp, i32]
    lib.jr_plan_set_palette.restype = ctypes.c_int
    lib.jr_plan_set_progress.argtypes = [vp, vp, vp]
    lib.jr_plan_set_progress.restype = ctypes.c_int
    lib.jr_set_image_schedule.argtypes = [i32, i32, i64, P(jr_schedule)]
    lib.jr_set_image_schedule.restype = ctypes.c_int
    lib.jr_get_image_schedule.argtypes = [i32, i32, i64, P(jr_schedule)]
    lib.jr_get_image_schedule.restype = ctypes.c_int
    lib.jr_clear_image_schedules.argtypes = []
    lib.jr_clear_image_schedules.restype = None
    lib.jr_plan_create.argtypes = [P(jr_frame), i32, vp, i64, P(jr_schedule), P(vp)]
    lib.jr_plan_create.restype = ctypes.c_int
    for name in ("jr_plan_launch", "jr_plan_capture", "jr_plan_replay"):
        getattr(lib, name).argtypes = [vp, vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.jr_plan_info.argtypes = [vp, P(i64), P(i32)]
    lib.jr_plan_info.restype = ctypes.c_int
    lib.jr_plan_destroy.argtypes = [vp]
    lib.jr_plan_destroy.restype = None
    lib.jr_get_default_schedule.argtypes = [i32, i32, P(jr_schedule)]
    lib.jr_get_default_schedule.restype = ctypes.c_int
    lib.jr_set_default_schedule.argtypes = [i32, P(jr_schedule)]
    lib.jr_set_default_schedule.restype = ctypes.c_int
    lib.jr_check_schedule.argtypes = [P(jr_schedule)]
    lib.jr_check_schedule.restype = ctypes.c_int
    lib.jr_check_frames.argtypes = [P(jr_frame), i32, i64]
    lib.jr_check_frames.restype = ctypes.c_int
    lib.jr_strerror.argtypes = [ctypes.c_int]
    lib.jr_strerror.restype = ctypes.c_char_p
    lib.jr_last_error_message.argtypes = []
    lib.jr_last_error_message.restype = ctypes.c_char_p
    lib.jr_device_info.argtypes = [P(i32), P(i64)]
    lib.jr_device_info.restype = ctypes.c_int
    lib.jr_shutdown.argtypes = []
    lib.jr_shutdown.restype = None
    return lib


lib = _load()


def _strerror(code: int) -> str:
    return lib.jr_strerror(code).decode()


def _check(rc: int):
    if rc != JR_OK:
        raise JuliaError(rc, lib.jr_last_error_message().decode())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _window(window) -> jr_window:
    return jr_window(*[float(v) for v in window])


def _out_tensor(out, shape):
    import torch
    if out is None:
        return torch.empty(shape, dtype=torch.int32, device="cuda")
    if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 CUDA tensor")
    if out.numel() < shape[0] * shape[1]:
        raise ValueError("out holds %d elements, need %d" % (out.numel(), shape[0] * shape[1]))
    return out


def _arena_tensor(arena, need: int, colours: bool = False):
    """Check a caller's output arena before its pointer and element count go
    to the library: a contiguous CUDA tensor of 32-bit elements (int32, or
    uint32 for colours) on the current device, holding at least `need`
    elements.  Anything else would hand the kernel a host address, a range
    shorter in bytes than its element count, or a strided view."""
    import torch
    ok = (torch.int32, torch.uint32) if colours else (torch.int32,)
    if not isinstance(arena, torch.Tensor) or arena.dtype not in ok:
        raise ValueError("arena must be an %s CUDA tensor" % "/".join(str(d) for d in ok))
    if not arena.is_cuda or not arena.is_contiguous():
        raise ValueError("arena must be a contiguous CUDA tensor")
    if arena.device.index != torch.cuda.current_device():
        raise ValueError("arena is on cuda:%d, the current device is cuda:%d"
                         % (arena.device.index, torch.cuda.current_device()))
    if arena.numel() < need:
        raise ValueError("arena holds %d elements, the frames need %d" % (arena.numel(), need))
    return arena


PALETTE_MAX = 8192  # JR_PALETTE_MAX


def _palette_ptr(palette):
    """(pointer, length) of a colour table: a 1-D contiguous int32 or uint32
    CUDA tensor of 1..PALETTE_MAX entries."""
    import torch
    if palette.dim() != 1 or not palette.is_cuda or not palette.is_contiguous() or \
            palette.dtype not in (torch.int32, torch.uint32):
        raise ValueError("palette must be a 1-D contiguous int32/uint32 CUDA tensor")
    if not 1 <= palette.numel() <= PALETTE_MAX:
        raise ValueError("palette holds %d entries, allowed 1..%d" % (palette.numel(), PALETTE_MAX))
    return ctypes.c_void_p(palette.data_ptr()), palette.numel()


_TUNED = None


def tuned_schedule(dtype: str, max_iter: int, pixels: int) -> Optional["Schedule"]:
    """The autotuner's schedule for this (dtype, cap, size) bucket on this
    device, from the shipped cache (autotune_cache.json), if it has one."""
    global _TUNED
    from . import autotune
    if _TUNED is None:
        try:
            _TUNED = autotune.load_cache()
        except (OSError, ValueError):
            _TUNED = {}
    key = (autotune.device_name(), dtype, autotune.cap_bucket(max_iter),
           autotune.pixel_bucket(pixels))
    if key not in _TUNED_MEMO:
        try:
            _TUNED_MEMO[key] = autotune.lookup(_TUNED, dtype, max_iter, pixels)
        except Exception:
            _TUNED_MEMO[key] = None
    return _TUNED_MEMO[key]


_TUNED_MEMO = {}
_IMAGE_SCHEDULES_DONE = False


def _install_image_schedules():
    """Hand the autotuner's single-image winners to the library
    (jr_set_image_schedule), once per process.  The library's table is
    process-wide and the library runs on gfx950 only, so the entries of the
    first device seen serve every device; later calls cost one test."""
    global _IMAGE_SCHEDULES_DONE
    if _IMAGE_SCHEDULES_DONE:
        return
    _IMAGE_SCHEDULES_DONE = True
    from . import autotune
    try:
        cache = autotune.load_cache()
    except (OSError, ValueError):
        return
    autotune.install_image_schedules(cache, autotune.device_name())


def image_schedule(dtype: str, max_iter: int, pixels: int) -> Schedule:
    """The schedule the library gives a one-image call of this size."""
    out = jr_schedule()
    _check(lib.jr_get_image_schedule(DTYPES[dtype], int(max_iter), int(pixels),
                                     ctypes.byref(out)))
    return Schedule.from_c(out)


def set_image_schedule(dtype: str, max_iter_limit: int, pixels_limit: int, schedule: Schedule):
    _check(lib.jr_set_image_schedule(DTYPES[dtype], int(max_iter_limit), int(pixels_limit),
                                     ctypes.byref(schedule.to_c())))


def render(c, window, width: int, height: int, max_iter: int, dtype: str = "fp64",
           out=None, stream=None, mode: str = "julia", plain: bool = False,
           schedule: Optional["Schedule"] = None, palette=None, degree: int = 2, lam=None):
    """Counts of one image as an int32 (height, width) CUDA tensor (row 0 = im_max).

    ``plain=True`` uses the one-thread-per-pixel comparator kernel.  Otherwise
    the schedule is ``schedule``, else the library's choice by size
    (julia_render / mandelbrot_render), which holds the autotuner's per-image
    winners (installed on first use, see _install_image_schedules).

    With ``palette`` (see _palette_ptr) each pixel holds the 32 bits of
    palette[min(count, len - 1)] instead of its count, stored by the kernel
    itself (julia_render_batch_colored).  ``degree`` 3..8 iterates the
    general map Z^degree + C (through julia_render_batch); with ``lam`` the
    map is the rational Z^degree + C + lam / Z^degree (Julia images, fp64 or
    fp32).
    """
    out = _out_tensor(out, (height, width))
    st = _stream_ptr(stream)
    dt = DTYPES[dtype]
    if (degree != 2 or lam is not None) and palette is None:
        if plain:
            schedule = Schedule(kernel="plain")
        f = _OneFrame(c, window, width, height, max_iter, dtype, mode, degree, lam)
        sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
        _check(lib.julia_render_batch(_frames_array([f], [0]), 1, ctypes.c_void_p(out.data_ptr()),
                                      width * height, sched, st))
        return out.view(-1)[: width * height].view(height, width)
    if palette is not None:
        pp, plen = _palette_ptr(palette)
        if plain:
            schedule = Schedule(kernel="plain")
        elif schedule is None and (mode != "julia" or degree != 2 or lam is not None):
            schedule = tuned_schedule(dtype, max_iter, width * height)
        if schedule is None and mode == "julia" and degree == 2 and lam is None:
            _install_image_schedules()
            c = complex(c)
            _check(lib.julia_render_colored(jr_complex(c.real, c.imag), _window(window), width,
                                            height, max_iter, dt, pp, plen,
                                            ctypes.c_void_p(out.data_ptr()), st))
        else:
            arr = _frames_array([_OneFrame(c, window, width, height, max_iter, dtype, mode,
                                           degree, lam)], [0])
            sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
            _check(lib.julia_render_batch_colored(arr, 1, pp, plen,
                                                  ctypes.c_void_p(out.data_ptr()),
                                                  width * height, sched, st))
        return out.view(-1)[: width * height].view(height, width)
    if not plain:
        if schedule is not None:
            f = _OneFrame(c, window, width, height, max_iter, dtype, mode)
            arr = _frames_array([f], [0])
            _check(lib.julia_render_batch(arr, 1, ctypes.c_void_p(out.data_ptr()),
                                          width * height, ctypes.byref(schedule.to_c()), st))
            return out.view(-1)[: width * height].view(height, width)
        # the library picks the schedule by size (jr_set_image_schedule)
        _install_image_schedules()
    if mode == "julia":
        c = complex(c)
        fn = lib.julia_render_plain if plain else lib.julia_render
        rc = fn(jr_complex(c.real, c.imag), _window(window), width, height, max_iter, dt,
                ctypes.c_void_p(out.data_ptr()), st)
    elif mode == "mandelbrot":
        fn = lib.mandelbrot_render_plain if plain else lib.mandelbrot_render
        rc = fn(_window(window), width, height, max_iter, dt, ctypes.c_void_p(out.data_ptr()), st)
    else:
        raise ValueError("mode must be 'julia' or 'mandelbrot'")
    _check(rc)
    return out.view(-1)[: width * height].view(height, width)


@dataclass
class _OneFrame:
    c: complex
    window: tuple
    width: int
    height: int
    max_iter: int
    dtype: str
    mode: str
    degree: int = 2
    lam: Optional[complex] = None


def _frames_array(frames, offsets, rows=None):
    """jr_frame records of objects with c, window, width, height, max_iter,
    dtype and optionally mode, degree and lam (a complex: the rational map
    Z^d + C + lam / Z^d)."""
    arr = (jr_frame * len(frames))()
    for k, f in enumerate(frames):
        c = complex(f.c)
        rb, re_ = (0, 0) if rows is None else rows[k]
        lam = getattr(f, "lam", None)
        lam_c = jr_complex(0.0, 0.0) if lam is None else jr_complex(complex(lam).real,
                                                                    complex(lam).imag)
        arr[k] = jr_frame(jr_complex(c.real, c.imag), _window(f.window), f.width, f.height,
                          f.max_iter, DTYPES[f.dtype], MODES[getattr(f, "mode", "julia")],
                          rb, re_, int(getattr(f, "degree", 2)), int(offsets[k]),
                          0 if lam is None else 1, 0, lam_c)
    return arr


def arena_layout(frames) -> Tuple[list, int]:
    """Element offsets of consecutive frames in one arena, and its size."""
    offs, total = [], 0
    for f in frames:
        offs.append(total)
        total += f.width * f.height
    return offs, total


def render_batch(frames: Sequence, schedule: Optional[Schedule] = None, arena=None,
                 offsets=None, stream=None, rows=None, palette=None):
    """Render frames (objects with c, window, width, height, max_iter, dtype, mode)
    in one persistent launch.  Returns (arena, views): views[k] is frame k's
    (height, width) counts inside the int32 arena, or with ``palette`` its
    colours (julia_render_batch_colored)."""
    import torch
    if offsets is None:
        offsets, total = arena_layout(frames)
    else:
        total = max(int(o) + f.width * f.height for o, f in zip(offsets, frames))
    if arena is None:
        arena = torch.empty(total, dtype=torch.int32, device="cuda")
    _arena_tensor(arena, total, colours=palette is not None)
    arr = _frames_array(frames, offsets, rows)
    sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
    if palette is not None:
        pp, plen = _palette_ptr(palette)
        rc = lib.julia_render_batch_colored(arr, len(frames), pp, plen,
                                            ctypes.c_void_p(arena.data_ptr()), arena.numel(),
                                            sched, _stream_ptr(stream))
    else:
        rc = lib.julia_render_batch(arr, len(frames), ctypes.c_void_p(arena.data_ptr()),
                                    arena.numel(), sched, _stream_ptr(stream))
    _check(rc)
    views = [arena[o: o + f.width * f.height].view(f.height, f.width)
             for o, f in zip(offsets, frames)]
    return arena, views


NOALLOC_MAX_FRAMES = 1024  # JR_NOALLOC_MAX_FRAMES


def render_batch_noalloc(frames: Sequence, arena, schedule: Optional[Schedule] = None,
                         offsets=None, stream=None):
    """render_batch through julia_render_batch_noalloc: the library allocates
    nothing for the call (its frame table and queue counters sit in a fixed
    device array, at most NOALLOC_MAX_FRAMES frames).  The caller provides the
    int32 arena; returns the frames' views into it.  Calls that overlap on one
    GPU share that array and race: keep them on one stream."""
    if offsets is None:
        offsets, total = arena_layout(frames)
    else:
        total = max(int(o) + f.width * f.height for o, f in zip(offsets, frames))
    _arena_tensor(arena, total)
    arr = _frames_array(frames, offsets)
    sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
    _check(lib.julia_render_batch_noalloc(arr, len(frames), ctypes.c_void_p(arena.data_ptr()),
                                          arena.numel(), sched, _stream_ptr(stream)))
    return [arena[o: o + f.width * f.height].view(f.height, f.width)
            for o, f in zip(offsets, frames)]


def render_cardioid_path(path: CardioidPath, schedule: Optional[Schedule] = None, arena=None,
                         stream=None):
    """All frames of a prescribed cardioid path in one call, their constants
    generated on the device (julia_render_cardioid_path).  Returns (arena,
    views) like render_batch."""
    import torch
    px = path.width * path.height
    if arena is None:
        arena = torch.empty(path.frames * px, dtype=torch.int32, device="cuda")
    _arena_tensor(arena, path.frames * px)
    sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
    _check(lib.julia_render_cardioid_path(ctypes.byref(path.to_c()),
                                          ctypes.c_void_p(arena.data_ptr()), arena.numel(),
                                          sched, _stream_ptr(stream)))
    return arena, [arena[k * px: (k + 1) * px].view(path.height, path.width)
                   for k in range(path.frames)]


class Plan:
    """A prepared batch: frame table uploaded once; launch() or a captured hipGraph."""

    @classmethod
    def cardioid(cls, path: CardioidPath, schedule: Optional[Schedule] = None, arena=None):
        """A plan over a prescribed cardioid path: every launch (and a
        captured graph) generates the frame table on the device, then renders
        it (jr_plan_create_cardioid)."""
        import torch
        self = cls.__new__(cls)
        self._h = None
        px = path.width * path.height
        self.arena = arena if arena is not None else torch.empty(path.frames * px,
                                                                 dtype=torch.int32, device="cuda")
        _arena_tensor(self.arena, path.frames * px)
        self.frames, self.offsets = [], [k * px for k in range(path.frames)]
        sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
        h = ctypes.c_void_p()
        _check(lib.jr_plan_create_cardioid(ctypes.byref(path.to_c()),
                                           ctypes.c_void_p(self.arena.data_ptr()),
                                           self.arena.numel(), sched, ctypes.byref(h)))
        self._h = h
        self.views = [self.arena[o: o + px].view(path.height, path.width) for o in self.offsets]
        self.frame_pixels = [px] * path.frames
        return self

    def __init__(self, frames: Sequence, schedule: Optional[Schedule] = None, arena=None,
                 offsets=None):
        import torch
        self._h = None
        if offsets is None:
            offsets, total = arena_layout(frames)
        else:
            total = max(int(o) + f.width * f.height for o, f in zip(offsets, frames))
        self.arena = arena if arena is not None else torch.empty(total, dtype=torch.int32,
                                                                 device="cuda")
        _arena_tensor(self.arena, total)
        self.frames = list(frames)
        self.offsets = list(offsets)
        arr = _frames_array(frames, offsets)
        sched = ctypes.byref(schedule.to_c()) if schedule is not None else None
        h = ctypes.c_void_p()
        _check(lib.jr_plan_create(arr, len(frames), ctypes.c_void_p(self.arena.data_ptr()),
                                  self.arena.numel(), sched, ctypes.byref(h)))
        self._h = h
        self.views = [self.arena[o: o + f.width * f.height].view(f.height, f.width)
                      for o, f in zip(self.offsets, self.frames)]
        self.frame_pixels = [f.width * f.height for f in self.frames]

    def launch(self, stream=None):
        _check(lib.jr_plan_launch(self._h, _stream_ptr(stream)))

    def capture(self, stream=None):
        _check(lib.jr_plan_capture(self._h, ctypes.c_void_p(0) if stream is None
                                   else _stream_ptr(stream)))

    def replay(self, stream=None):
        _check(lib.jr_plan_replay(self._h, _stream_ptr(stream)))

    def set_palette(self, palette=None):
        """Store colours from ``palette`` (None: counts) in later launches; a
        captured graph is dropped and must be captured again."""
        if palette is None:
            _check(lib.jr_plan_set_palette(self._h, None, 0))
        else:
            pp, plen = _palette_ptr(palette)
            _check(lib.jr_plan_set_palette(self._h, pp, plen))
        self.palette = palette  # keep the table alive while the plan may use it

    def set_progress(self, done=None, stop=None):
        """Per-frame done counters and a stop flag for later launches
        (jr_plan_set_progress): ``done`` an int32 CUDA tensor of one counter
        per frame, ``stop`` None or an int32 tensor of one element (on the
        device, or pinned host memory that the host may set while a launch
        runs).  None, None turns progress off.  A captured graph is dropped."""
        import torch
        for t, name, n in ((done, "done", len(self.frame_pixels)), (stop, "stop", 1)):
            if t is None:
                continue
            if t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < n:
                raise ValueError("%s: a contiguous int32 tensor of at least %d elements" % (name, n))
            if name == "done" and not t.is_cuda:
                raise ValueError("done: a device tensor")
            if name == "stop" and not (t.is_cuda or t.is_pinned()):
                raise ValueError("stop: a device tensor or pinned host memory")
        _check(lib.jr_plan_set_progress(self._h,
                                        None if done is None else ctypes.c_void_p(done.data_ptr()),
                                        None if stop is None else ctypes.c_void_p(stop.data_ptr())))
        self.progress = (done, stop)  # keep them alive while launches may use them

    def incomplete(self, done):
        """Indices of the frames whose counter (host copy of ``done``) falls
        short of their pixel count."""
        d = [int(v) for v in done]
        return [k for k, px in enumerate(self.frame_pixels) if d[k] != px]

    def info(self):
        t, w = ctypes.c_int64(), ctypes.c_int32()
        _check(lib.jr_plan_info(self._h, ctypes.byref(t), ctypes.byref(w)))
        return {"tiles": t.value, "workgroups": w.value}

    def close(self):
        if self._h:
            lib.jr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_schedule(dtype: str, max_iter: int = 100) -> Schedule:
    s = jr_schedule()
    _check(lib.jr_get_default_schedule(DTYPES[dtype], max_iter, ctypes.byref(s)))
    return Schedule.from_c(s)


def set_default_schedule(dtype: str, schedule: Schedule):
    _check(lib.jr_set_default_schedule(DTYPES[dtype], ctypes.byref(schedule.to_c())))


def check_schedule(schedule: Schedule) -> int:
    return lib.jr_check_schedule(ctypes.byref(schedule.to_c()))


def check_frames(frames, offsets, capacity: int, rows=None) -> int:
    arr = _frames_array(frames, offsets, rows)
    return lib.jr_check_frames(arr, len(frames), capacity)


def device_info():
    n, m = ctypes.c_int32(), ctypes.c_int64()
    _check(lib.jr_device_info(ctypes.byref(n), ctypes.byref(m)))
    return {"num_cus": n.value, "hbm_bytes": m.value}


def last_error() -> str:
    return lib.jr_last_error_message().decode()
