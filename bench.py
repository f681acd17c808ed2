"""Benchmark of the escape-time hot path on one MI355X.

Workload (a step): the single-image 4096x4096 configuration -- window
[-1.6, 1.6]^2, C = 0.7885 exp(i theta) with theta from seeds 0..3, caps 100
and 1000 -- rendered in FP32 with the tuned persistent kernel, one launch per
image (8 images per step).  Inputs are synthetic and live in HBM before the
timed region; nothing leaves the device inside it.

Metric: useful pixel-iterations per second (sum of the output counts over the
step / step time), in Gpixel-iter/s.  One pixel-iteration is 8 flops
(x^2, y^2, x^2+y^2, x^2-y^2, +Re C, 2x, (2x)y, +Im C).

The JSON line also carries the roofline of the dominant kernel (useful FLOP/s
of the persistent kernel from HIP events around each launch, against the
vector FP32 peak), the single-threaded CPU oracle on a bounded sample of the
same workload, and further legs in "extra": FP64, the plain one-thread-per-
pixel kernel on the same images, the 256-frame 1920x1080 parameter path in
one persistent launch, and the 512x512 FP64 image's latency.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
PEAK_HBM_GBS = 8000.0
FLOP_PER_ITER = 8


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="bound on the CPU-oracle sample")
    p.add_argument("--no-extra", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    return p.parse_args()


def frames_single_4096(dtype):
    import workloads as wl
    return [wl.single_4096(seed, it, dtype) for it in (100, 1000) for seed in range(4)]


def time_renders(jr, torch, frames, outs, steps, warmup, plain=False):
    """Time `steps` passes; each pass renders every frame with one launch.
    Returns (ms per step, per-launch kernel ms list from events)."""
    def one_pass(events=None):
        for k, (f, o) in enumerate(zip(frames, outs)):
            if events is not None:
                events[k][0].record()
            jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=o, plain=plain)
            if events is not None:
                events[k][1].record()

    for _ in range(warmup):
        one_pass()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in frames] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        one_pass(ev[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = sum(a.elapsed_time(b) for row in ev for a, b in row) / steps
    return (t1 - t0) * 1e3 / steps, kernel_ms


def cpu_baseline(frames, seconds):
    """The oracle, single-threaded, on rows spread over the step's images until
    `seconds` of CPU work; returns pixel-iter/s and the sample description."""
    import numpy as np
    import oracle
    t_end = time.perf_counter() + seconds
    total_iters, total_px, elapsed = 0, 0, 0.0
    rows_done = 0
    stride = 64
    rng_rows = [list(range(r, f.height, stride)) for f in frames for r in (0,)]
    k = 0
    while time.perf_counter() < t_end and rows_done < sum(len(r) for r in rng_rows):
        for fi, f in enumerate(frames):
            if k >= len(rng_rows[fi]):
                continue
            j = rng_rows[fi][k]
            ii = np.arange(f.width, dtype=np.int32)
            jj = np.full(f.width, j, dtype=np.int32)
            t0 = time.perf_counter()
            c = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
            elapsed += time.perf_counter() - t0
            total_iters += int(c.sum(dtype=np.int64))
            total_px += f.width
            rows_done += 1
        k += 1
    return total_iters / elapsed, ("every %dth row of each of the %d images, first %d rows "
                                   "(%d pixels, %.1f s single-threaded)"
                                   % (stride, len(frames), rows_done, total_px, elapsed))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported "
              "(the path needs no exchange between GPUs; see DESIGN.md on sharding)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1611_03079_amd as jr
    import workloads as wl

    torch.cuda.set_device(0)
    frames = frames_single_4096("fp32")
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in frames]
    ms_step, kernel_ms = time_renders(jr, torch, frames, outs, args.steps, args.warmup)
    iters = sum(int(o.sum(dtype=torch.int64).item()) for o in outs)
    pixels = sum(f.pixels for f in frames)
    value = iters / (ms_step * 1e-3) / 1e9
    achieved_tflops = FLOP_PER_ITER * iters / (kernel_ms * 1e-3) / 1e12

    line = {
        "metric": "Gpixel-iters/s (FP64/FP32/float-float) vs plain kernel; p99 frame latency",
        "value": round(value, 3),
        "unit": "Gpixel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single_4096: 4096x4096, window [-1.6,1.6]^2, "
                               "C=0.7885exp(i theta(seed)), seeds 0-3, max_iter {100,1000}, "
                               "FP32, tuned persistent kernel, one launch per image",
                   "images_per_step": len(frames), "pixels_per_step": pixels,
                   "pixel_iters_per_step": iters,
                   "schedule": jr.default_schedule("fp32").__dict__},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "jr_persistent<unroll, FP32>",
                     "kernel_ms_per_step": round(kernel_ms, 4)},
    }
    extra = {}
    if not args.no_extra:
        steps = max(3, args.steps // 4)
        # plain kernel on the same images
        ms_plain, k_plain = time_renders(jr, torch, frames, outs, steps, 1, plain=True)
        extra["fp32_plain"] = {"gpixel_iter_s": round(iters / (ms_plain * 1e-3) / 1e9, 3),
                               "ms_per_step": round(ms_plain, 4)}
        extra["fp32_tuned_vs_plain"] = round(ms_plain / ms_step, 3)
        f64 = frames_single_4096("fp64")
        ms64, k64 = time_renders(jr, torch, f64, outs, steps, 1)
        it64 = sum(int(o.sum(dtype=torch.int64).item()) for o in outs)
        ms64p, _ = time_renders(jr, torch, f64, outs, steps, 1, plain=True)
        extra["fp64"] = {"gpixel_iter_s": round(it64 / (ms64 * 1e-3) / 1e9, 3),
                         "ms_per_step": round(ms64, 4),
                         "frac_fp64_peak": round(FLOP_PER_ITER * it64 / (k64 * 1e-3) / 1e12
                                                 / PEAK_FP64_TFLOPS, 4),
                         "plain_gpixel_iter_s": round(it64 / (ms64p * 1e-3) / 1e9, 3)}
        del outs
        # batched parameter path, one persistent launch per pass
        pp = wl.parameter_path()
        plan = jr.Plan(pp, jr.default_schedule("fp32"))
        plan.capture()
        for _ in range(2):
            plan.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(3, args.steps // 4)
        e0.record()
        for _ in range(reps):
            plan.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_pp = e0.elapsed_time(e1) / reps
        it_pp = int(plan.arena.sum(dtype=torch.int64).item())
        px_pp = sum(f.pixels for f in pp)
        extra["parameter_path_256x1920x1080_fp32"] = {
            "gpixel_iter_s": round(it_pp / (ms_pp * 1e-3) / 1e9, 3),
            "ms_per_batch": round(ms_pp, 4),
            "frac_fp32_peak": round(FLOP_PER_ITER * it_pp / (ms_pp * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "store_gb_s": round(4 * px_pp / (ms_pp * 1e-3) / 1e9, 1),
            "pixel_iters": it_pp, "pixels": px_pp}
        plan.close()
        # 512x512 FP64 latency (launch-bound)
        o = torch.empty((512, 512), dtype=torch.int32, device="cuda")
        f1 = wl.single_512()
        for _ in range(5):
            jr.render(f1.c, f1.window, 512, 512, 100, "fp64", out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            jr.render(f1.c, f1.window, 512, 512, 100, "fp64", out=o)
            torch.cuda.synchronize()
        extra["single_512_fp64_latency_us"] = round((time.perf_counter() - t0) / 50 * 1e6, 1)
        line["extra"] = extra
    if not args.no_cpu:
        rate, sample = cpu_baseline(frames, args.cpu_seconds)
        line["cpu_baseline"] = {"value": round(rate / 1e9, 5), "unit": "Gpixel-iter/s",
                                "cores": 1, "kind": "oracle", "sample": sample}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
