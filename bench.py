"""Benchmark of the escape-time hot path on one MI355X.

Workload (one step): the batched parameter path -- 256 frames of 1920x1080,
C_k = 0.7885 exp(2 pi i k / 256), window Re[-1.78, 1.78] x Im[-1, 1], cap 100,
FP32 -- rendered in ONE launch with the autotuned kernel and schedule,
replayed from a captured hipGraph.  This is the batched form the throughput
target is quoted on.  Inputs are synthetic and resident in HBM before the timed
region; nothing leaves the device inside it.

Metric: useful pixel-iterations per second (sum of the output counts over the
step / step time), in Gpixel-iter/s.  A pixel-iteration is 8 flops (x^2, y^2,
x^2+y^2, x^2-y^2, +Re C, 2x, (2x)y, +Im C); 4 bytes are written per pixel and
nothing is read.

The JSON line also carries the roofline of the kernel (HIP events around each
launch on the stream it runs on), the single-threaded CPU oracle on a bounded
sample of the same workload, and further legs in "extra":
  - the plain one-thread-per-pixel kernel on the same frames, the
    persistent-queue mode, and the fused colour store;
  - the single 4096x4096 images in FP32 and FP64, and the 512x512 FP64
    image's latency;
  - the 1024-frame uneven batch (FP32 and float-float, one launch);
  - a batch of the general map Z^3 + C;
  - the square-image sweep of the paper's timing study, GPU beside the CPU
    oracle;
  - the serving loop's p50/p99 latency under Poisson arrivals;
  - the FP32 and float-float pixel fractions that differ from FP64.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32: 256 CU x 2.4 GHz x 256 flop/clk
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64: 256 CU x 2.4 GHz x 128 flop/clk
# FP32 without packed instructions (the build leaves them off): one FMA per
# lane per clock, 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
FLOP_PER_ITER = 8
BYTES_PER_PIXEL = 4
METRIC = "Gpixel-iters/s (FP64/FP32/float-float) vs plain kernel; p99 frame latency"

# HBM bytes per launch of the headline kernel from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE (KiB summed over a dispatch), scaled by what the same
# counters read for a device copy of 1 GiB (fetch x2.0, write x1.0), keyed by
# the kernel instance they were taken on.  The summaries with their commands
# are in profiles/.  A kernel without an entry reports null.
MEASURED_TRAFFIC_BYTES = {
    "jr_rows<8, 2, 1>": 2199092400,  # 620,544 B fetched + 2,198,471,856 B written
    "jr_tiled<8, 0, 2, 0>": 2124197256,  # 662,559 B fetched + 2,123,534,697 B written
}

# The kernel instance a schedule launches for an FP32-only batch that stores
# counts (template arguments as rocprofv3 prints them).
def kernel_instance(sched):
    if sched.kernel == "rows":
        # one-wave workgroups for dispatched tiles, four waves with the queues
        return "jr_rows<%d, 2, %d>" % (sched.unroll, 4 if sched.persistent else 1)
    if sched.kernel == "plain":
        return "jr_plain_batch<2>"
    return "jr_tiled<%d, %d, 2, %d>" % (sched.unroll, sched.defer, int(sched.kernel == "hybrid"))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-extra", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=2.5)
    p.add_argument("--schedule", choices=("tuned", "plain", "tiled"), default="tuned",
                   help="headline schedule: the autotuned one (default), the batched "
                        "one-thread-per-pixel kernel, or the refill stream (64x64 tiles, "
                        "counted blocks of 8), for profiling comparisons")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run an elementwise device copy of 1 GiB (read 1 GiB, write 1 GiB) "
                        "whose FETCH_SIZE / WRITE_SIZE counters calibrate the traffic figures")
    return p.parse_args()


def tuned_schedule(jr, name, frames):
    """Schedule from the committed autotune cache, else tuned here (minutes)."""
    from paper_1611_03079_amd import autotune as at
    cache = at.load_cache()
    e = cache.get("_workloads", {}).get(name)
    if e:
        return jr.Schedule(**e["schedule"]), "cache"
    print("bench: no autotune cache entry for %s; tuning it first (minutes)" % name,
          file=sys.stderr, flush=True)
    best, _, _ = at.tune(frames, reps=3, verbose=True)
    return best, "tuned at start"


def time_plan_steps(torch, plan, steps, warmup, graph=True):
    """ms per step (wall, synchronised) and mean kernel ms (events)."""
    run = plan.replay if graph else plan.launch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        run()
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms = sum(a.elapsed_time(b) for a, b in ev) / steps
    return (t1 - t0) * 1e3 / steps, kms


def time_renders(jr, torch, frames, outs, reps, plain):
    def one():
        for f, o in zip(frames, outs):
            jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=o,
                      plain=plain, mode=f.mode)
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def count_sum(torch, views):
    return sum(int(v.sum(dtype=torch.int64).item()) for v in views)


def cpu_baseline(frames, seconds):
    """The oracle, single-threaded, on whole rows taken in a fixed interleaved
    order (row j of every frame, rows stepping by 7 through the image), until
    `seconds` of CPU work."""
    import numpy as np
    import oracle
    H = frames[0].height
    rows = [(3 + 7 * m) % H for m in range(H)]  # 7 and 1080 are coprime: every row once
    picks = [(fi, j) for j in rows for fi in range(len(frames))]
    iters = px = 0
    spent = 0.0
    done = 0
    for fi, j in picks:
        if spent >= seconds:
            break
        f = frames[fi]
        ii = np.arange(f.width, dtype=np.int32)
        jj = np.full(f.width, j, dtype=np.int32)
        t0 = time.perf_counter()
        c = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        spent += time.perf_counter() - t0
        iters += int(c.sum(dtype=np.int64))
        px += f.width
        done += 1
    sample = ("%d whole 1920-pixel rows (%d pixels): rows j = 3, 10, 17, ... (step 7 mod "
              "1080) of all 256 frames in turn, oracle FP32 formulation, %.1f s "
              "single-threaded" % (done, px, spent))
    return iters / spent, sample


def extra_legs(args, torch, jr, wl, frames, sched, ms_headline, iters):
    from paper_1611_03079_amd.serve import GpuBackend, Server, run_open_loop
    ex = {}
    reps = 3
    # plain kernel: one launch per frame, same frames
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in frames]
    ms_plain = time_renders(jr, torch, frames, outs, reps, plain=True)
    ex["parameter_path_plain_per_frame"] = {
        "gpixel_iter_s": round(iters / (ms_plain * 1e-3) / 1e9, 2), "ms_per_step": round(ms_plain, 4)}
    ex["tuned_batch_vs_plain"] = round(ms_plain / ms_headline, 3)
    del outs
    # persistent work-queue mode of the same batch
    from dataclasses import replace
    pers = replace(sched, persistent=1, waves_per_cu=32)
    plan = jr.Plan(frames, pers)
    ms_p, _ = time_plan_steps(torch, plan, 5, 1, graph=False)
    plan.close()
    ex["parameter_path_persistent_queues"] = {"ms_per_step": round(ms_p, 4),
                                              "gpixel_iter_s": round(iters / (ms_p * 1e-3) / 1e9, 2)}
    # fused colour store: the same batch storing colours from a 101-entry table
    import numpy as np
    pal = torch.from_numpy(np.random.default_rng(0).integers(
        0, 2 ** 31, size=101, dtype=np.int64).astype(np.int32)).cuda()
    # counts timed right beside the colours, so that the ratio compares the
    # two under the same clock
    plan = jr.Plan(frames, sched)
    plan.capture()
    ms_n, _ = time_plan_steps(torch, plan, 10, 2, graph=True)
    plan.set_palette(pal)
    plan.capture()
    ms_c, kms_c = time_plan_steps(torch, plan, 10, 2, graph=True)
    plan.close()
    ex["parameter_path_colour_store"] = {
        "ms_per_step": round(ms_c, 4), "kernel_ms": round(kms_c, 4),
        "palette_entries": 101, "counts_ms_per_step_beside": round(ms_n, 4),
        "counts_over_colours_time": round(ms_n / ms_c, 3)}
    # single 4096x4096 images, FP32 and FP64, tuned vs plain
    for dt in ("fp32", "fp64"):
        fr = [wl.single_4096(s, it, dt) for it in (100, 1000) for s in range(4)]
        outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in fr]
        ms_t = time_renders(jr, torch, fr, outs, reps, plain=False)
        it_s = count_sum(torch, outs)
        ms_pl = time_renders(jr, torch, fr, outs, reps, plain=True)
        peak = PEAK_FP32_TFLOPS if dt == "fp32" else PEAK_FP64_TFLOPS
        ex["single_4096_%s" % dt] = {
            "gpixel_iter_s": round(it_s / (ms_t * 1e-3) / 1e9, 2),
            "plain_gpixel_iter_s": round(it_s / (ms_pl * 1e-3) / 1e9, 2),
            "frac_vector_peak": round(FLOP_PER_ITER * it_s / (ms_t * 1e-3) / 1e12 / peak, 4),
            "images": len(fr), "pixel_iters": it_s}
        del outs
    # 512x512 FP64: launch-bound latency, tuned and plain
    f1 = wl.single_512("fp64")
    o = torch.empty((512, 512), dtype=torch.int32, device="cuda")
    for plain in (False, True):
        for _ in range(5):
            jr.render(f1.c, f1.window, 512, 512, 100, "fp64", out=o, plain=plain)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            jr.render(f1.c, f1.window, 512, 512, 100, "fp64", out=o, plain=plain)
            torch.cuda.synchronize()
        ex["single_512_fp64_latency_us_" + ("plain" if plain else "tuned")] = round(
            (time.perf_counter() - t0) / 50 * 1e6, 1)
    # uneven batch: 1024 FP32 and float-float frames of random sides (256..4096)
    # and caps, one launch into a 24.5 GB arena; the plain kernel then renders
    # the same frames one launch each into the same arena
    ub = wl.uneven_batch(0, n=1024)
    usched, _ = tuned_schedule(jr, "uneven_fp32_ff", ub)
    plan = jr.Plan(ub, usched)
    ms_u, _ = time_plan_steps(torch, plan, 1, 1, graph=False)
    it_u = count_sum(torch, plan.views)
    ms_up = time_renders(jr, torch, ub, plan.views, 1, plain=True)
    plan.close()
    del plan
    torch.cuda.empty_cache()
    ex["uneven_batch_1024_frames_fp32_ff"] = {
        "gpixel_iter_s": round(it_u / (ms_u * 1e-3) / 1e9, 2), "ms": round(ms_u, 3),
        "plain_per_frame_ms": round(ms_up, 3), "vs_plain": round(ms_up / ms_u, 3),
        "frames": len(ub), "pixels": sum(f.pixels for f in ub), "pixel_iters": it_u,
        "schedule": usched.__dict__}
    # general map Z^3 + C: 32 frames of 1920x1080, one launch, against the
    # plain kernel launched per frame
    gp = wl.general_path(32, 3)
    gsched, _ = tuned_schedule(jr, "general_deg3_fp32", gp)
    plan = jr.Plan(gp, gsched)
    ms_g, _ = time_plan_steps(torch, plan, 5, 1, graph=False)
    it_g = count_sum(torch, plan.views)
    plan.close()
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in gp]

    def plain_general():
        for f, o in zip(gp, outs):
            jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=o, plain=True,
                      degree=3)
    plain_general()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_general()
    torch.cuda.synchronize()
    ms_gp = (time.perf_counter() - t0) * 1e3
    del outs
    ex["general_map_degree3_32_frames_fp32"] = {
        "gpixel_iter_s": round(it_g / (ms_g * 1e-3) / 1e9, 2), "ms": round(ms_g, 3),
        "plain_per_frame_ms": round(ms_gp, 3), "vs_plain": round(ms_gp / ms_g, 3),
        "schedule": gsched.__dict__, "pixel_iters": it_g}
    # serving: Poisson arrivals at several rates, with the precision policy
    # as specified (float-float for mid widths) and with FP64 for every window
    # narrower than FP32 handles (on MI355X FP64 runs at the FP32 rate)
    from paper_1611_03079_amd.serve import PrecisionPolicy
    serve = {}
    policies = {"ff_mid": PrecisionPolicy(), "fp64_narrow": PrecisionPolicy(ff_min_width=float("inf"))}
    for pname, rates in (("ff_mid", (50, 200, 800, 2000)), ("fp64_narrow", (200, 2000))):
        for rate in rates:
            n = max(20, int(rate * args.serve_seconds))
            reqs = wl.serving_stream(11, float(rate), n)
            cap = 8 * 1920 * 1080
            srv = Server(GpuBackend(cap), cap, step_budget=2.0e8, copy_out=False,
                         policy=policies[pname])
            st = run_open_loop(srv, reqs, drain_timeout=5.0)
            torch.cuda.synchronize()
            span = max(st.t_last - st.t_first, 1e-9)
            serve["%s_rate_%d" % (pname, rate)] = {
                "offered": n, "completed": st.completed,
                "p50_ms": round(st.percentile(50) * 1e3, 2), "p99_ms": round(st.percentile(99) * 1e3, 2),
                "completed_req_s": round(st.completed / span, 1), "steps": st.steps}
            del srv
            torch.cuda.empty_cache()
    ex["serving"] = serve
    # the paper's timing study (Figure 1): square images of side 10 .. 10000,
    # C = -0.8 + 0.156i, window [-1.5, 1.5]^2, cap 100, FP64: GPU time per
    # image (tuned and plain, synchronised, launch included) beside the
    # single-threaded oracle on this host (sides up to 3162)
    if not args.no_cpu:
        import oracle
    sweep = {}
    for f in wl.square_sweep("fp64"):
        o = torch.empty((f.height, f.width), dtype=torch.int32, device="cuda")
        row = {}
        for plain in (False, True):
            jr.render(f.c, f.window, f.width, f.height, 100, "fp64", out=o, plain=plain)
            torch.cuda.synchronize()
            reps = 20 if f.width <= 1000 else 5
            t0 = time.perf_counter()
            for _ in range(reps):
                jr.render(f.c, f.window, f.width, f.height, 100, "fp64", out=o, plain=plain)
            torch.cuda.synchronize()
            row["gpu_plain_ms" if plain else "gpu_tuned_ms"] = round(
                (time.perf_counter() - t0) * 1e3 / reps, 4)
        if not args.no_cpu and f.width <= 3162:
            t0 = time.perf_counter()
            oracle.render(f.c, f.window, f.width, f.height, 100, "fp64")
            row["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        sweep["side_%d" % f.width] = row
        del o
    ex["figure1_square_sweep_fp64"] = sweep
    # pixels whose FP32 / float-float count differs from FP64 (GPU vs GPU)
    mism = {}
    for dt in ("fp32", "ff"):
        diff = tot = 0
        for f in frames[::32]:
            a = jr.render(f.c, f.window, f.width, f.height, f.max_iter, "fp64")
            b = jr.render(f.c, f.window, f.width, f.height, f.max_iter, dt)
            diff += int((a != b).sum().item())
            tot += f.pixels
        mism[dt] = round(diff / tot, 6)
    ex["mismatch_vs_fp64_parameter_path"] = mism
    return ex


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported: the path has no "
              "exchange between GPUs (DESIGN.md describes how it would shard)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1611_03079_amd as jr
    import workloads as wl

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    frames = wl.parameter_path()
    if args.schedule == "plain":
        sched, sched_src = jr.Schedule(kernel="plain"), "--schedule plain"
    elif args.schedule == "tiled":
        sched, sched_src = jr.Schedule(64, 64, 8, 0, 32, 0, 16, "cost"), "--schedule tiled"
    else:
        sched, sched_src = tuned_schedule(jr, "parameter_path_fp32", frames)
    plan = jr.Plan(frames, sched)
    plan.capture()
    ms_step, kernel_ms = time_plan_steps(torch, plan, args.steps, args.warmup, graph=True)
    iters = count_sum(torch, plan.views)
    info = plan.info()
    plan.close()
    pixels = sum(f.pixels for f in frames)
    value = iters / (ms_step * 1e-3) / 1e9
    store_gbs = BYTES_PER_PIXEL * pixels / (kernel_ms * 1e-3) / 1e9
    alu_tflops = FLOP_PER_ITER * iters / (kernel_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
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
        "config": {"workload": "parameter_path: 256 frames 1920x1080, C=0.7885exp(2 pi i k/256), "
                               "window Re[-1.78,1.78] x Im[-1,1], max_iter 100, FP32, one launch "
                               "per step (hipGraph replay) with the schedule below",
                   "frames": len(frames), "pixels_per_step": pixels, "pixel_iters_per_step": iters,
                   "schedule": sched.__dict__, "schedule_source": sched_src,
                   "tiles": info["tiles"], "workgroups": info["workgroups"]},
        "roofline": {"bound": "hbm", "achieved": round(store_gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(store_gbs / PEAK_HBM_GBS, 4),
                     "traffic": MEASURED_TRAFFIC_BYTES.get(kernel_instance(sched)),
                     "algorithmic_bytes_per_launch": BYTES_PER_PIXEL * pixels,
                     "kernel_ms": round(kernel_ms, 4),
                     "alu": {"achieved": round(alu_tflops, 2), "peak": PEAK_FP32_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(alu_tflops / PEAK_FP32_TFLOPS, 4),
                             "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                             "frac_unpacked": round(alu_tflops / PEAK_FP32_UNPACKED_TFLOPS, 4),
                             "flops_per_launch": FLOP_PER_ITER * iters},
                     "kernel": kernel_instance(sched) + " (libjulia.so)"},
    }
    if not args.no_extra:
        line["extra"] = extra_legs(args, torch, jr, wl, frames, sched, ms_step, iters)
    if not args.no_cpu:
        rate, sample = cpu_baseline(frames, args.cpu_seconds)
        line["cpu_baseline"] = {"value": round(rate / 1e9, 5), "unit": "Gpixel-iter/s",
                                "cores": 1, "kind": "oracle", "sample": sample}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
