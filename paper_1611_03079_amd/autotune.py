"""Autotuner for the tiled kernel's schedule.

A schedule (tile shape, iteration block length and escape-test mode, refill
threshold, persistent or one-wave-per-tile, resident waves, frame order)
never changes a count: only which lane computes which pixel and when.  The
tuner therefore times candidate schedules on a representative batch with HIP
events around prepared launches (jr_plan_launch) and keeps the fastest.

Search, in stages from a base schedule:
  1. the iteration block (unroll, defer),
  2. tile shape x scheduling mode x refill threshold, then the tile order
     (frames as given, or the most expensive first),
  3. resident waves per compute unit (persistent mode only),
  4. the iteration block again under the chosen tiling,
  5. the hybrid stream (fresh packets tested every iteration, survivors
     refilled) under that tiling, for several bail points,
  6. the two-phase row-packet kernel: its first block, then scheduling mode,
     refill, resident waves and tile shape, then the tile order, then its
     first block again, then its drain's blocks (counted or deferred),
  7. the batched one-thread-per-pixel kernel, in both tile orders, as the
     last candidates.
A workload too large to search whole is searched on a subset of its frames;
``confirm`` then times the subset's best candidates on the whole workload and
keeps the fastest there.

Results are cached in a JSON file keyed by (device, dtype, cap bucket, pixel
bucket); ``apply_cache`` installs the cached winners as the library defaults
(jr_set_default_schedule), which julia_render and julia_render_batch use when
no schedule is passed.
"""
import json
import math
import os
import time
from dataclasses import asdict, replace
from typing import Dict, List, Optional, Sequence, Tuple

import paper_1611_03079_amd as jr

BLOCKS = [(1, 0), (2, 0), (4, 0), (8, 0), (4, 1), (8, 1), (16, 1)]
TILES = [(64, 1), (64, 4), (64, 16), (32, 8), (16, 16), (64, 64)]
REFILLS = [8, 16, 32, 64]
WAVES = [8, 16, 24, 32]
HYBRID_BAILS = [4, 8, 16, 32]
ROWS_FIRST = [4, 8, 12, 16, 20, 24, 32, 48, 64]
ROWS_HANDOFF = [0, 16, 32, 64, 96, 128, 160, 192]
ORDERS = [dict(order="table"), dict(order="cost")]

DEFAULT_CACHE = os.environ.get(
    "JR_AUTOTUNE_CACHE",
    os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json"))


def cap_bucket(max_iter: int) -> str:
    return "cap<=128" if max_iter <= 128 else "cap<=1024" if max_iter <= 1024 else "cap>1024"


PIXEL_EDGES = [("px<16K", 1 << 14), ("px<64K", 1 << 16), ("px<512K", 1 << 19),
               ("px<4M", 1 << 22), ("px<64M", 64 << 20)]


def pixel_bucket(pixels: int) -> str:
    for name, edge in PIXEL_EDGES:
        if pixels < edge:
            return name
    return "px>=64M"


def cache_key(device: str, dtype: str, max_iter: int, pixels: int, batch: bool = False) -> str:
    """Bucket of a single image, or (batch) of a batch launch: batches are
    filed apart so that a batch's winner never serves one image."""
    parts = [device, dtype, cap_bucket(max_iter), pixel_bucket(pixels)]
    return "|".join(parts + (["batch"] if batch else []))


# Below this many pixels a render() call's host work and launch outweigh its
# kernel: such images are timed as their caller waits for them, by the wall
# clock over back-to-back render() calls.
WALL_PIXELS = 1 << 16


def time_singles(frames, schedule: jr.Schedule, reps: int = 3) -> float:
    """Sum over the frames of the time of each rendered on its own.  A single
    image under a plain schedule runs the two-dimensional one-thread-per-pixel
    kernel (julia_render_plain), which is what is timed for it.  Images below
    WALL_PIXELS are timed by time_render_wall."""
    if all(f.pixels < WALL_PIXELS for f in frames):
        return sum(time_render_wall(f, schedule, reps=reps) for f in frames)
    if schedule.kernel == "plain":
        return sum(time_render_plain(f, reps=reps) for f in frames)
    return sum(time_plan([f], schedule, reps=reps) for f in frames)


def time_render_wall(f, schedule: jr.Schedule, reps: int = 3, calls: int = 50) -> float:
    """Wall time (ms) per render() call of one frame under `schedule`: the
    median over `reps` runs of `calls` back-to-back calls, synchronised once
    at the end of each run (host work, launch and kernel)."""
    import torch
    out = torch.empty((f.height, f.width), dtype=torch.int32, device="cuda")
    plain = schedule.kernel == "plain"

    def one():
        jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=out,
                  plain=plain, schedule=None if plain else schedule, mode=f.mode,
                  degree=f.degree)

    one()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for _ in range(calls):
            one()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3 / calls)
    times.sort()
    return times[len(times) // 2]


def time_render_plain(f, reps: int = 3, span_ms: float = 5.0) -> float:
    """Sustained device time (ms) per render of one frame by the plain kernel,
    timed like time_plan."""
    import torch
    out = torch.empty((f.height, f.width), dtype=torch.int32, device="cuda")

    def one():
        jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=out,
                  plain=True, mode=f.mode, degree=f.degree)

    one()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    one()
    b.record()
    b.synchronize()
    n = int(min(200, max(1, math.ceil(span_ms / max(a.elapsed_time(b), 1e-3)))))
    times = []
    for _ in range(reps):
        a.record()
        for _ in range(n):
            one()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / n)
    times.sort()
    return times[len(times) // 2]


def time_plan(frames, schedule: jr.Schedule, reps: int = 3, warmup: int = 1,
              span_ms: float = 5.0) -> float:
    """Device time (ms) per launch of `frames` under `schedule`, sustained:
    the median over `reps` runs of back-to-back launches, each run at least
    `span_ms` long.  The chip's clock under a steady load, not a lone
    launch's, decides throughput, and the two can rank schedules
    differently."""
    import torch
    plan = jr.Plan(frames, schedule)
    try:
        for _ in range(warmup):
            plan.launch()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.launch()
        b.record()
        b.synchronize()
        n = int(min(200, max(1, math.ceil(span_ms / max(a.elapsed_time(b), 1e-3)))))
        times = []
        for _ in range(reps):
            a.record()
            for _ in range(n):
                plan.launch()
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b) / n)
        times.sort()
        return times[len(times) // 2]
    finally:
        plan.close()


def _time(frames, s, reps, singles):
    return time_singles(frames, s, reps) if singles else time_plan(frames, s, reps=reps)


def _stage(frames, base: jr.Schedule, variants: List[dict], reps: int, log: list,
           singles: bool = False) -> jr.Schedule:
    best, best_t = base, math.inf
    seen = set()
    for v in variants:
        s = replace(base, **v)
        if s in seen or jr.check_schedule(s) != jr.JR_OK:
            continue
        seen.add(s)
        t = _time(frames, s, reps, singles)
        log.append((asdict(s), t))
        if t < best_t:
            best, best_t = s, t
    return best


class _ProgressLog(list):
    """A tuning log that reports every 16th candidate on stderr."""

    def __init__(self, base):
        super().__init__(base)

    def append(self, item):
        super().append(item)
        if len(self) % 16 == 0:
            import sys
            d, t = item
            print("autotune: %d candidates, last %s/%dx%d %.4f ms" % (
                len(self), d["kernel"], d["tile_w"], d["tile_h"], t), file=sys.stderr, flush=True)


def tune(frames: Sequence, base: Optional[jr.Schedule] = None, reps: int = 3,
         log: Optional[list] = None, singles: bool = False,
         verbose: bool = False) -> Tuple[jr.Schedule, float, list]:
    """Search schedules for `frames`; returns (best, its median ms, log).
    With ``singles`` each frame is timed as a launch of its own (the way
    single images are rendered) and the times are summed.  ``verbose`` prints
    a line to stderr after every stage."""
    log = [] if log is None else log
    if verbose:
        log = _ProgressLog(log)
    base = base or jr.Schedule()
    s = _stage(frames, base, [dict(unroll=u, defer=d) for u, d in BLOCKS], reps, log, singles)
    s = _stage(frames, s, [dict(tile_w=tw, tile_h=th, persistent=p, refill=r)
                           for tw, th in TILES for p in (1, 0) for r in REFILLS], reps, log,
               singles)
    s = _stage(frames, s, ORDERS, reps, log, singles)
    if s.persistent:
        s = _stage(frames, s, [dict(waves_per_cu=w) for w in WAVES], reps, log, singles)
    # re-check the block choice under the final tiling
    s = _stage(frames, s, [dict(unroll=u, defer=d) for u, d in BLOCKS], reps, log, singles)
    best_t = min(t for d, t in log if jr.Schedule(**d) == s)
    # the hybrid stream under the chosen tiling, with several bail points
    tiled = s
    for bail in HYBRID_BAILS:
        h = replace(tiled, kernel="hybrid", bail=bail)
        t = _time(frames, h, reps, singles)
        log.append((asdict(h), t))
        if t < best_t:
            s, best_t = h, t
    # the two-phase row-packet kernel: first-block length x second block,
    # then scheduling mode, refill and resident waves, then the first block
    # again with the pairs' handoff point
    r = jr.Schedule(64, 8, 8, 0, 16, 1, 32, s.order, "rows", 4)
    r = _stage(frames, r, [dict(bail=p, unroll=k) for p in ROWS_FIRST for k in (4, 8)], reps, log,
               singles)
    r = _stage(frames, r, [dict(persistent=p, refill=rf, waves_per_cu=w, tile_w=tw, tile_h=th)
                           for p in (1, 0) for rf in (8, 16, 32) for w in (16, 32)
                           for tw, th in ((64, 8), (64, 16), (64, 32), (64, 64), (32, 16))],
               reps, log, singles)
    r = _stage(frames, r, ORDERS, reps, log, singles)
    r = _stage(frames, r, [dict(bail=p, handoff=h) for p in ROWS_FIRST for h in ROWS_HANDOFF],
               reps, log, singles)
    # the drain's blocks: counted, or testing their last iterate
    r = _stage(frames, r, [dict(defer=d, unroll=k) for d in (0, 1) for k in (4, 8)], reps, log,
               singles)
    t = min(tt for d, tt in log if jr.Schedule(**d) == r)
    if t < best_t:
        s, best_t = r, t
    # the one-thread-per-pixel kernel over the batch is a candidate too
    for order in ("table", "cost"):
        plain = jr.Schedule(kernel="plain", order=order)
        t = _time(frames, plain, reps, singles)
        log.append((asdict(plain), t))
        if t < best_t:
            s, best_t = plain, t
    return s, best_t, log


def confirm(frames: Sequence, log: list, top: int = 6, reps: int = 2,
            singles: bool = False) -> Tuple[jr.Schedule, float, list]:
    """Times the `top` fastest distinct schedules of a tuning log (taken on a
    subset of a workload), each also in the other tile order, on `frames`
    (the whole workload); returns the fastest there, its time and the
    timings."""
    ranked = []
    for d, t in sorted(log, key=lambda e: e[1]):
        sc = jr.Schedule(**d)
        if sc not in ranked:
            ranked.append(sc)
        if len(ranked) == top:
            break
    cands = []
    for sc in ranked:
        for o in ("cost", "table"):
            v = replace(sc, order=o)
            if v not in cands:
                cands.append(v)
    timings = [(asdict(v), _time(frames, v, reps, singles)) for v in cands]
    d, t = min(timings, key=lambda e: e[1])
    return jr.Schedule(**d), t, timings


_DEVICE_NAMES: Dict[int, str] = {}


def device_name() -> str:
    import torch
    d = torch.cuda.current_device()
    if d not in _DEVICE_NAMES:
        p = torch.cuda.get_device_properties(d)
        _DEVICE_NAMES[d] = getattr(p, "gcnArchName", p.name).split(":")[0]
    return _DEVICE_NAMES[d]


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(cache: Dict[str, dict], path: str = DEFAULT_CACHE):
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def record(cache: Dict[str, dict], frames: Sequence, schedule: jr.Schedule, ms: float,
           singles: bool = False):
    """File the winner under the bucket its launches fall in: the batch, or
    with ``singles`` one of its frames."""
    dtype = max(set(f.dtype for f in frames), key=lambda d: sum(f.pixels for f in frames if f.dtype == d))
    cap = max(f.max_iter for f in frames)
    px = max(f.pixels for f in frames) if singles else sum(f.pixels for f in frames)
    cache[cache_key(device_name(), dtype, cap, px, batch=not singles)] = {
        "schedule": asdict(schedule), "ms": ms}


def lookup(cache: Dict[str, dict], dtype: str, max_iter: int, pixels: int) -> Optional[jr.Schedule]:
    e = cache.get(cache_key(device_name(), dtype, max_iter, pixels))
    return jr.Schedule(**e["schedule"]) if e else None


CAP_LIMITS = {"cap<=128": 128, "cap<=1024": 1024, "cap>1024": 2 ** 31 - 1}
PIXEL_LIMITS = dict([(name, edge - 1) for name, edge in PIXEL_EDGES] + [("px>=64M", 2 ** 63 - 1)])


def install_image_schedules(cache: Dict[str, dict], device: str) -> int:
    """Install the single-image buckets of `device` from the cache as the
    library's per-size schedules (jr_set_image_schedule); returns how many."""
    n = 0
    for key, e in cache.items():
        parts = key.split("|")
        if len(parts) != 4 or parts[0] != device:
            continue  # batch entries and other devices
        _, dtype, cap, px = parts
        if cap not in CAP_LIMITS or px not in PIXEL_LIMITS:
            continue  # a bucket of an older layout
        jr.set_image_schedule(dtype, CAP_LIMITS[cap], PIXEL_LIMITS[px],
                              jr.Schedule(**e["schedule"]))
        n += 1
    return n


def apply_cache(cache: Dict[str, dict], max_iter: int = 100, pixels: int = 1 << 24):
    """Install cached schedules for (dtype, max_iter, pixels) as library defaults."""
    for dt in ("fp64", "fp32", "ff"):
        s = lookup(cache, dt, max_iter, pixels)
        if s is not None:
            jr.set_default_schedule(dt, s)


# ------------------------------------------------------------------ command line
# workloads rendered one image per launch (tuned and filed per image)
SINGLES = {"single_4096_fp32_cap100", "single_4096_fp32_cap1000", "single_4096_fp64_cap100",
           "single_4096_fp64_cap1000", "single_512_fp64", "single_tiny_fp64", "single_small_fp64",
           "single_1000_fp64", "single_10000_fp64", "single_512_fp32", "single_tiny_fp32",
           "single_small_fp32", "single_1000_fp32", "single_10000_fp32"}


def standard_workloads():
    """Representative workloads the library is tuned for: batches rendered in
    one launch, and single images (SINGLES) rendered one per launch."""
    import workloads as wl
    return {
        "parameter_path_fp32": wl.parameter_path(),
        "parameter_path_fp64": wl.parameter_path(dtype="fp64"),
        "parameter_path_ff": wl.parameter_path(dtype="ff"),
        "single_4096_fp32_cap100": [wl.single_4096(s, 100, "fp32") for s in range(2)],
        "single_4096_fp32_cap1000": [wl.single_4096(s, 1000, "fp32") for s in range(2)],
        "single_4096_fp64_cap100": [wl.single_4096(s, 100, "fp64") for s in range(2)],
        "single_4096_fp64_cap1000": [wl.single_4096(s, 1000, "fp64") for s in range(2)],
        "single_512_fp64": [wl.single_512("fp64")],
        # the other sizes of the square sweep, one pixel bucket each
        "single_tiny_fp64": wl.square_sweep("fp64", sides=(10, 32, 100)),
        "single_small_fp64": wl.square_sweep("fp64", sides=(200,)),
        "single_1000_fp64": wl.square_sweep("fp64", sides=(1000, 2000)),
        "single_10000_fp64": wl.square_sweep("fp64", sides=(10000,)),
        # the same sizes in FP32: without them FP32 images below 4M pixels
        # would take the 4096^2 images' schedule
        "single_512_fp32": [wl.single_512("fp32")],
        "single_tiny_fp32": wl.square_sweep("fp32", sides=(10, 32, 100)),
        "single_small_fp32": wl.square_sweep("fp32", sides=(200,)),
        "single_1000_fp32": wl.square_sweep("fp32", sides=(1000, 2000)),
        "single_10000_fp32": wl.square_sweep("fp32", sides=(10000,)),
        # searched on its first 64 frames, confirmed on all 1024 (CONFIRM)
        "uneven_fp32_ff": wl.uneven_batch(0, n=64),
        "cardioid_path_fp32": wl.cardioid_path(64),
        "general_deg3_fp32": wl.general_path(32, 3),
        "rational_deg2_fp32": wl.rational_path(32, 2, dtype="fp32"),
        "rational_deg2_fp64": wl.rational_path(32, 2, dtype="fp64"),
        "mandelbrot_zoom_fp64": wl.mandelbrot_zoom(64),
    }


# workloads searched on a subset and confirmed on the whole workload
CONFIRM = {"uneven_fp32_ff": lambda: __import__("workloads").uneven_batch(0, n=1024)}


def main(argv=None):
    import argparse
    import torch
    p = argparse.ArgumentParser(description="tune schedules and write the cache")
    p.add_argument("--out", default=DEFAULT_CACHE)
    p.add_argument("--only", nargs="*")
    p.add_argument("--reps", type=int, default=3)
    args = p.parse_args(argv)
    torch.cuda.set_device(0)
    cache = load_cache(args.out)
    for name, frames in standard_workloads().items():
        if args.only and name not in args.only:
            continue
        singles = name in SINGLES
        print("autotune: %s (%d frames)" % (name, len(frames)), flush=True)
        best, ms, log = tune(frames, reps=args.reps, singles=singles, verbose=True)
        record(cache, frames, best, ms, singles=singles)
        entry = {"schedule": asdict(best), "ms": ms, "candidates": len(log)}
        if name in CONFIRM:
            whole = CONFIRM[name]()
            subset_best = best
            best, ms_whole, timings = confirm(whole, log)
            entry = {"schedule": asdict(best), "ms": ms_whole, "candidates": len(log),
                     "searched_on_frames": len(frames), "confirmed_on_frames": len(whole),
                     "subset_winner": asdict(subset_best),
                     "subset_winner_ms_whole": min(t for d, t in timings
                                                   if jr.Schedule(**d) == subset_best),
                     "confirmed": [[d, t] for d, t in timings]}
            print("%-22s confirmed on %d frames: %9.4f ms  %s" % (name, len(whole), ms_whole,
                                                                  best), flush=True)
        cache.setdefault("_workloads", {})[name] = entry
        print("%-22s %9.4f ms  %s" % (name, ms, best), flush=True)
        save_cache(cache, args.out)


if __name__ == "__main__":
    main()
