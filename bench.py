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
  - the parameter path in FP64 and in float-float, and Section 3's
    prescribed cardioid path with its constants generated on the device;
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

PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1611_03079_amd", "csrc", "julia_kernels.hip")


def kernel_source_sha256():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel: str, workload: str, schedule: dict):
    """HBM bytes per launch of `kernel` on `workload` under `schedule` from
    the rocprofv3 FETCH_SIZE / WRITE_SIZE summaries in profiles/: a summary
    states
        traffic_bytes_per_launch: <workload> | <kernel> | <schedule json> | <bytes>
        kernel_source_sha256: <hash of julia_kernels.hip the counters ran on>
    Returns (bytes, file) when a summary matches the kernel, the workload, the
    schedule and the current kernel source; (None, reason) otherwise, so that
    a kernel or schedule changed since its counters were taken reports no
    traffic."""
    if not os.path.isdir(PROFILES):
        return None, "no profiles/ folder"
    now = kernel_source_sha256()
    stale = None
    for name in sorted(os.listdir(PROFILES)):
        entries, sha = [], None
        with open(os.path.join(PROFILES, name), errors="replace") as f:
            for line in f:
                if line.startswith("traffic_bytes_per_launch:"):
                    entries.append([x.strip() for x in line.split(":", 1)[1].split("|")])
                elif line.startswith("kernel_source_sha256:"):
                    sha = line.split(":", 1)[1].strip()
        for e in entries:
            if len(e) != 4:
                continue
            wl_name, kern, sched_json, nbytes = e
            if wl_name == workload and kern == kernel and json.loads(sched_json) == schedule:
                if sha == now:
                    return int(nbytes), "profiles/" + name
                stale = "profiles/%s was taken on another kernel source" % name
    return None, stale or "no counters for %s on %s in profiles/" % (kernel, workload)

# The kernel instance a schedule launches for an FP32-only batch that stores
# counts (template arguments as rocprofv3 prints them).
def kernel_instance(sched):
    if sched.kernel == "rows":
        # one-wave workgroups for dispatched tiles, four waves with the queues;
        # the last argument: deferred drain blocks
        return "jr_rows<%d, 2, %d, %d>" % (sched.unroll, 4 if sched.persistent else 1,
                                           1 if sched.defer else 0)
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
    p.add_argument("--serve-seconds", type=float, default=20.0,
                   help="longest arrival window per serving rate (s); a rate also stops "
                        "after --serve-requests requests")
    p.add_argument("--serve-requests", type=int, default=5000)
    p.add_argument("--schedule", choices=("tuned", "plain", "tiled"), default="tuned",
                   help="headline schedule: the autotuned one (default), the batched "
                        "one-thread-per-pixel kernel, or the refill stream (64x64 tiles, "
                        "counted blocks of 8), for profiling comparisons")
    p.add_argument("--leg", choices=("headline", "single_4096_fp64", "single_4096_fp32",
                                      "parameter_path_fp64", "parameter_path_ff", "figure1"),
                   default="headline",
                   help="run one workload alone (for profiling): the 8 single 4096^2 "
                        "images (seeds 0..3, caps 100 and 1000) rendered one call each, "
                        "tuned or with --plain; or a parameter path in FP64 / float-float "
                        "in one launch per step (autotuned schedule, or --plain); or the timing "
                        "study of square images (figure1)")
    p.add_argument("--plain", action="store_true",
                   help="with --leg: the one-thread-per-pixel comparator kernel")
    p.add_argument("--leg-schedule", default=None,
                   help="with --leg: this schedule (a JSON object of Schedule fields) "
                        "instead of the autotuned one, for every call of the leg")
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


def tuned_schedule_or_default(jr, name):
    """Schedule from the committed autotune cache, else None (the library's
    default for the batch's dtype)."""
    from paper_1611_03079_amd import autotune as at
    e = at.load_cache().get("_workloads", {}).get(name)
    if e:
        return jr.Schedule(**e["schedule"]), "cache"
    return None, "library default"


def serving_sweep(args, torch, wl):
    from paper_1611_03079_amd.serve import GpuBackend, PrecisionPolicy, Server, run_open_loop
    out = {}
    policies = (("calibrated", PrecisionPolicy(), (50, 100, 200, 500, 1000, 2000, 4000)),
                ("three_way_ff", PrecisionPolicy.specified(), (50, 200, 1000, 2000)))
    for pname, pol, rates in policies:
        sat = None
        for rate in rates:
            n = max(20, min(args.serve_requests, int(rate * args.serve_seconds)))
            reqs = wl.serving_stream(11, float(rate), n)
            cap = 8 * 1920 * 1080
            srv = Server(GpuBackend(cap), cap, copy_out=False, policy=pol)
            st = run_open_loop(srv, reqs, drain_timeout=5.0)
            torch.cuda.synchronize()
            span = max(st.t_last - st.t_first, 1e-9)
            dts = {}
            for r in reqs:
                dts[r.frame.dtype] = dts.get(r.frame.dtype, 0) + 1
            kept_up = (not st.saturated) and st.completed / span >= 0.9 * rate
            if kept_up:
                sat = rate
            out["%s_rate_%d" % (pname, rate)] = {
                "offered": n, "completed": st.completed, "unfinished": len(st.unfinished),
                "seconds": round(reqs[-1].arrival_s, 2),
                "p50_ms": round(st.percentile(50) * 1e3, 2),
                "p99_ms": round(st.percentile(99) * 1e3, 2),
                "completed_req_s": round(st.completed / span, 1), "steps": st.steps,
                "kept_up": kept_up, "dtypes": dts,
                "learnt_rate_units_per_s": float("%.3g" % srv.rate.rate)}
            del srv
            torch.cuda.empty_cache()
            print("bench: serving %s at %d req/s: p99 %.1f ms, %s" % (
                pname, rate, st.percentile(99) * 1e3, "kept up" if kept_up else "saturated"),
                file=sys.stderr, flush=True)
            if not kept_up:
                break   # higher rates only queue longer
        out["%s_highest_rate_kept_up" % pname] = sat
    return out


SETTLE_S = 0.5


def settle_clocks(torch, plan, seconds=SETTLE_S):
    """Replays the step, untimed, for `seconds` before the warm-up steps.  The
    GPU raises its clock over the first tens of milliseconds of sustained
    load (a profile of 23 back-to-back launches ran 1.26 ms at first and
    0.92 ms at the end), so without this the timed steps would measure the
    ramp.  Returns the settle time in ms."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            plan.replay()
        torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


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


def time_renders(jr, torch, frames, outs, reps, plain, schedule=None):
    def one():
        for f, o in zip(frames, outs):
            jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=o,
                      plain=plain, mode=f.mode, schedule=schedule)
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def count_sum(torch, views):
    return sum(int(v.sum(dtype=torch.int64).item()) for v in views)


ROWS_PER_CALL = 8


def _row_picks(frames):
    """Whole rows in a fixed interleaved order: rows step by 7 through the
    image (7 and 1080 are coprime, so every row comes once), taken
    ROWS_PER_CALL at a time, each group from every frame in turn."""
    H = frames[0].height
    rows = [(3 + 7 * m) % H for m in range(H)]
    groups = [rows[k: k + ROWS_PER_CALL] for k in range(0, H, ROWS_PER_CALL)]
    return [(fi, g) for g in groups for fi in range(len(frames))]


def _oracle_rows(job):
    """Worker: the oracle on the row groups picks[start::step] (one oracle
    call per group) until `seconds` pass; returns (pixel-iterations, pixels,
    rows, seconds spent)."""
    import numpy as np
    import oracle
    frames, picks, start, step, seconds = job
    iters = px = done = 0
    t0 = time.perf_counter()
    for fi, rows in picks[start::step]:
        if time.perf_counter() - t0 >= seconds:
            break
        f = frames[fi]
        ii = np.tile(np.arange(f.width, dtype=np.int32), len(rows))
        jj = np.repeat(np.asarray(rows, dtype=np.int32), f.width)
        c = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        iters += int(c.sum(dtype=np.int64))
        px += ii.size
        done += len(rows)
    return iters, px, done, time.perf_counter() - t0


def host_cpu():
    """The host's CPU model (lscpu / /proc/cpuinfo), its logical CPUs and the
    CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, os.cpu_count(), allowed


def uneven_cpu_sample(frames, per_frame=128):
    """The single-threaded oracle on a deterministic sample of the uneven
    batch: `per_frame` pixels of every frame (positions from a generator
    seeded by the frame's index), each frame's sample time scaled by its
    pixel count over the sample's, summed: the extrapolated time of the whole
    batch on one core, labelled as extrapolated.  Uses the oracle's own
    counts only."""
    import numpy as np
    import oracle
    t, it, whole = {}, {}, 0.0
    for k, f in enumerate(frames):
        rng = np.random.default_rng(k)
        ii = rng.integers(0, f.width, per_frame).astype(np.int32)
        jj = rng.integers(0, f.height, per_frame).astype(np.int32)
        t0 = time.perf_counter()
        c = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        dt_s = time.perf_counter() - t0
        t[f.dtype] = t.get(f.dtype, 0.0) + dt_s
        it[f.dtype] = it.get(f.dtype, 0) + int(c.sum(dtype=np.int64))
        whole += dt_s * f.pixels / per_frame
    return {"sample": "%d pixels of each of the %d frames, single thread" % (per_frame, len(frames)),
            "sample_seconds": round(sum(t.values()), 2),
            "rate_gpixel_iter_s_by_dtype": {dt: round(it[dt] / t[dt] / 1e9, 4) for dt in t},
            "whole_batch_seconds_one_core_extrapolated": round(whole, 1),
            "extrapolated": True}


def cpu_baseline(frames, seconds):
    """The oracle on whole rows of the headline workload (FP32 formulation):
    single-threaded for `seconds`, then one host thread per core (at most 16,
    the host share of one GPU), each calling the same single-threaded oracle
    on every n-th row of the same order, for `seconds` of wall time.  The
    oracle library releases the interpreter lock while it runs, so the
    threads run in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    picks = _row_picks(frames)
    it1, px1, rows1, s1 = _oracle_rows((frames, picks, 0, 1, seconds))
    model, ncpu, allowed = host_cpu()
    n = max(1, min(16, allowed))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(n) as pool:
        res = list(pool.map(_oracle_rows, [(frames, picks, k, n, seconds) for k in range(n)]))
    wall = time.perf_counter() - t0
    busy = max(r[3] for r in res)
    itn = sum(r[0] for r in res)
    return {
        "single": (it1 / s1, "%d whole 1920-pixel rows (%d pixels): rows j = 3, 10, 17, ... "
                   "(step 7 mod 1080) in groups of %d, each group from all 256 frames in "
                   "turn, one oracle call per group, oracle FP32 formulation, %.1f s on one "
                   "core" % (rows1, px1, ROWS_PER_CALL, s1)),
        "all": (itn / busy, n, "the same row order dealt round-robin to %d threads, each "
                "calling the single-threaded oracle, %d rows (%d pixels), %.1f s of wall time "
                "(%.1f s with start-up)" % (n, sum(r[2] for r in res), sum(r[1] for r in res),
                                             busy, wall)),
        "cpu_model": model, "nproc": ncpu, "cpus_allowed": allowed,
    }


def extra_legs(args, torch, jr, wl, frames, sched, ms_headline, iters):
    ex = {}
    reps = 3
    # plain kernel: one launch per frame, same frames
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in frames]
    ms_plain = time_renders(jr, torch, frames, outs, reps, plain=True)
    ex["parameter_path_plain_per_frame"] = {
        "gpixel_iter_s": round(iters / (ms_plain * 1e-3) / 1e9, 2), "ms_per_step": round(ms_plain, 4)}
    ex["tuned_batch_vs_plain"] = round(ms_plain / ms_headline, 3)
    del outs
    # the same frames in FP64 and in float-float, one launch each (library
    # default schedule of the dtype), beside the plain kernel per frame
    for dt in ("fp64", "ff"):
        fr = wl.parameter_path(dtype=dt)
        dsched, dsrc = tuned_schedule_or_default(jr, "parameter_path_" + dt)
        plan = jr.Plan(fr, dsched)
        plan.capture()
        settle_clocks(torch, plan, 0.3)
        ms_d, kms_d = time_plan_steps(torch, plan, 10, 2, graph=True)
        it_d = count_sum(torch, plan.views)
        info_d = plan.info()
        plan.close()
        outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in fr]
        ms_dp = time_renders(jr, torch, fr, outs, 1, plain=True)
        del outs
        # float-float counts its useful flops against the FP32 vector peak
        # (its hardware operation count is in profiles/)
        peak = PEAK_FP64_TFLOPS if dt == "fp64" else PEAK_FP32_TFLOPS
        useful_tf = FLOP_PER_ITER * it_d / (kms_d * 1e-3) / 1e12
        ex["parameter_path_%s" % dt] = {
            "gpixel_iter_s": round(it_d / (ms_d * 1e-3) / 1e9, 2), "ms_per_step": round(ms_d, 4),
            "kernel_ms": round(kms_d, 4), "pixel_iters": it_d,
            "plain_per_frame_ms": round(ms_dp, 4), "vs_plain": round(ms_dp / ms_d, 3),
            "useful_flop_frac_of_peak": round(useful_tf / peak, 4), "peak_tflops": peak,
            "schedule": (dsched.__dict__ if dsched else dsrc),
            "workgroups": info_d["workgroups"]}
        if dt == "ff":
            ex["parameter_path_ff"]["useful_flop_frac_of_unpacked_fp32"] = round(
                useful_tf / PEAK_FP32_UNPACKED_TFLOPS, 4)
    # Section 3's prescribed path with a growing cardioid: 256 frames of
    # 1920x1080, four trips of 64 frames while a goes from 3.9 to 3.5, FP32,
    # cap 100; the constants are generated on the device in every step (one
    # graph holds the generator and the render), beside per-frame launches of
    # the plain kernel with the same constants formed on the host (libm)
    g = wl.growing_cardioid_path()
    path = jr.CardioidPath(g.step, g.a0, g.da, g.window, g.frames, g.width, g.height,
                           g.max_iter, g.dtype)
    csched, csrc = tuned_schedule_or_default(jr, "cardioid_path_fp32")
    plan = jr.Plan.cardioid(path, csched)
    plan.capture()
    ms_cd, kms_cd = time_plan_steps(torch, plan, 10, 2, graph=True)
    it_cd = count_sum(torch, plan.views)
    plan.close()
    import math
    host = [wl.Frame(wl.cardioid_point(2.0 * math.pi * k / 64, g.a0 - g.da * k), g.window,
                     g.width, g.height, g.max_iter, g.dtype) for k in range(g.frames)]
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in host]
    ms_cp = time_renders(jr, torch, host, outs, 1, plain=True)
    it_cp = count_sum(torch, outs)
    del outs
    ex["cardioid_path_device_generated_fp32"] = {
        "gpixel_iter_s": round(it_cd / (ms_cd * 1e-3) / 1e9, 2), "ms_per_step": round(ms_cd, 4),
        "kernel_ms": round(kms_cd, 4), "pixel_iters": it_cd, "frames": g.frames,
        "a0": g.a0, "a_last": round(g.a0 - g.da * (g.frames - 1), 6),
        "schedule": csched.__dict__ if csched else csrc,
        "plain_per_frame_host_constants_ms": round(ms_cp, 4),
        "plain_gpixel_iter_s": round(it_cp / (ms_cp * 1e-3) / 1e9, 2),
        "vs_plain": round(ms_cp / ms_cd, 3)}
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
        # each image alone (seed, cap): its mean count and both rates
        per = {}
        for k, (f, o) in enumerate(zip(fr, outs)):
            t_t = time_renders(jr, torch, [f], [o], reps, plain=False)
            it_f = int(o.sum(dtype=torch.int64).item())
            t_p = time_renders(jr, torch, [f], [o], reps, plain=True)
            per["seed%d_cap%d" % (k % 4, f.max_iter)] = {
                "mean_count": round(it_f / f.pixels, 3), "tuned_ms": round(t_t, 4),
                "plain_ms": round(t_p, 4),
                "gpixel_iter_s": round(it_f / (t_t * 1e-3) / 1e9, 1),
                "plain_gpixel_iter_s": round(it_f / (t_p * 1e-3) / 1e9, 1)}
        ex["single_4096_%s" % dt] = {
            "gpixel_iter_s": round(it_s / (ms_t * 1e-3) / 1e9, 2),
            "plain_gpixel_iter_s": round(it_s / (ms_pl * 1e-3) / 1e9, 2),
            "frac_vector_peak": round(FLOP_PER_ITER * it_s / (ms_t * 1e-3) / 1e12 / peak, 4),
            "images": len(fr), "pixel_iters": it_s, "per_image": per}
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
    it_dt = {}
    for f, v in zip(ub, plan.views):
        it_dt[f.dtype] = it_dt.get(f.dtype, 0) + int(v.sum(dtype=torch.int64).item())
    it_u = sum(it_dt.values())
    ms_up = time_renders(jr, torch, ub, plan.views, 1, plain=True)
    plan.close()
    del plan
    torch.cuda.empty_cache()
    ex["uneven_batch_1024_frames_fp32_ff"] = {
        "gpixel_iter_s": round(it_u / (ms_u * 1e-3) / 1e9, 2), "ms": round(ms_u, 3),
        "plain_per_frame_ms": round(ms_up, 3), "vs_plain": round(ms_up / ms_u, 3),
        "frames": len(ub), "pixels": sum(f.pixels for f in ub), "pixel_iters": it_u,
        "pixel_iters_by_dtype": it_dt, "schedule": usched.__dict__}
    if not args.no_cpu:
        ex["uneven_batch_1024_frames_fp32_ff"]["cpu_oracle_extrapolated"] = \
            uneven_cpu_sample(ub)
    # general map Z^3 + C: 32 frames of 1920x1080, one launch, against the
    # plain kernel launched per frame
    gp = wl.general_path(32, 3)
    gsched, _ = tuned_schedule(jr, "general_deg3_fp32", gp)
    plan = jr.Plan(gp, gsched)
    plan.capture()
    settle_clocks(torch, plan, 0.3)
    ms_g, _ = time_plan_steps(torch, plan, 10, 2, graph=True)
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
    # rational two-parameter maps Z^2 + C + lam / Z^2: 32 frames of 1920x1080
    # along the parameter path's circle, FP32 and FP64, one launch against
    # the plain kernel launched per frame
    for dt in ("fp32", "fp64"):
        rp = wl.rational_path(32, 2, dtype=dt)
        rsched, rsrc = tuned_schedule_or_default(jr, "rational_deg2_" + dt)
        plan = jr.Plan(rp, rsched)
        plan.capture()
        settle_clocks(torch, plan, 0.3)
        ms_r, _ = time_plan_steps(torch, plan, 10, 2, graph=True)
        it_r = count_sum(torch, plan.views)
        plan.close()
        outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in rp]

        def plain_rational():
            for f, o in zip(rp, outs):
                jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, out=o,
                          plain=True, degree=2, lam=f.lam)
        plain_rational()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain_rational()
        torch.cuda.synchronize()
        ms_rp = (time.perf_counter() - t0) * 1e3
        del outs
        ex["rational_map_degree2_32_frames_" + dt] = {
            "gpixel_iter_s": round(it_r / (ms_r * 1e-3) / 1e9, 2), "ms": round(ms_r, 3),
            "plain_per_frame_ms": round(ms_rp, 3), "vs_plain": round(ms_rp / ms_r, 3),
            "schedule": (rsched.__dict__ if rsched else rsrc), "pixel_iters": it_r}
    # Mandelbrot zoom (Section 3): 64 frames of 1920x1080, the window from 3
    # down to 1e-5 wide around a boundary point, cap 1000, FP64, one launch
    # against the plain kernel launched per frame
    mz = wl.mandelbrot_zoom(64)
    msched, msrc = tuned_schedule_or_default(jr, "mandelbrot_zoom_fp64")
    plan = jr.Plan(mz, msched)
    plan.capture()
    settle_clocks(torch, plan, 0.3)
    ms_m, kms_m = time_plan_steps(torch, plan, 10, 2, graph=True)
    it_m = count_sum(torch, plan.views)
    plan.close()
    outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in mz]
    ms_mp = time_renders(jr, torch, mz, outs, 1, plain=True)
    del outs
    ex["mandelbrot_zoom_64_frames_fp64"] = {
        "gpixel_iter_s": round(it_m / (ms_m * 1e-3) / 1e9, 2), "ms": round(ms_m, 3),
        "kernel_ms": round(kms_m, 3), "plain_per_frame_ms": round(ms_mp, 3),
        "vs_plain": round(ms_mp / ms_m, 3),
        "useful_flop_frac_of_peak": round(FLOP_PER_ITER * it_m / (kms_m * 1e-3) / 1e12
                                          / PEAK_FP64_TFLOPS, 4),
        "schedule": (msched.__dict__ if msched else msrc), "pixel_iters": it_m}
    # serving: open-loop Poisson arrivals at the specified rates, each for
    # --serve-seconds or --serve-requests requests, whichever ends first,
    # with the calibrated precision policy (FP32 where it stays within 0.5%
    # of FP64, FP64 elsewhere) and with the three-way policy (float-float
    # between 1e-5 and the FP32 region); the step budget is learnt from
    # measured step times (2 ms target).  Unfinished requests count in the
    # percentiles at the latency they had when the run was cut off.
    ex["serving"] = serving_sweep(args, torch, wl)
    # the paper's timing study (Figure 1): square images of side 10 .. 10000,
    # C = -0.8 + 0.156i, window [-1.5, 1.5]^2, cap 100, FP64 and FP32: GPU
    # time per image (tuned and plain, synchronised, launch included) beside
    # the single-threaded oracle on this host in the same arithmetic
    ex.update(figure1_sweep(args, torch, jr, wl))
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


def figure1_sweep(args, torch, jr, wl):
    """The paper's timing study (Figure 1): wall time per render() call of
    square images, tuned and plain, each the median of five runs of
    back-to-back calls synchronised at the end (launch and host work
    included), beside the single-threaded oracle in the same arithmetic."""
    if not args.no_cpu:
        import oracle
        oracle.render(0j, (-1.0, 1.0, -1.0, 1.0), 2, 2, 1, "fp64")  # load it before timing
    ex = {}
    for dt in ("fp64", "fp32"):
        sweep = {}
        for f in wl.square_sweep(dt):
            o = torch.empty((f.height, f.width), dtype=torch.int32, device="cuda")
            row = {}
            for plain in (False, True):
                jr.render(f.c, f.window, f.width, f.height, 100, dt, out=o, plain=plain)
                torch.cuda.synchronize()
                reps = 20 if f.width <= 1000 else 5
                runs = []
                for _ in range(5):
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        jr.render(f.c, f.window, f.width, f.height, 100, dt, out=o, plain=plain)
                    torch.cuda.synchronize()
                    runs.append((time.perf_counter() - t0) * 1e3 / reps)
                row["gpu_plain_ms" if plain else "gpu_tuned_ms"] = round(sorted(runs)[2], 4)
            if not args.no_cpu:
                t0 = time.perf_counter()
                oracle.render(f.c, f.window, f.width, f.height, 100, dt)
                row["cpu_oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
            sweep["side_%d" % f.width] = row
            del o
        ex["figure1_square_sweep_%s" % dt] = sweep
    return ex


def run_leg(args, torch, jr, wl):
    """One workload alone, for profiling: `steps` timed repetitions after
    `warmup`; prints one JSON line with its rate."""
    forced = None
    if args.leg_schedule is not None:
        if args.plain:
            sys.exit("--leg-schedule and --plain exclude each other")
        forced = jr.Schedule(**json.loads(args.leg_schedule))
    if args.leg == "figure1":
        print(json.dumps({"leg": "figure1", **figure1_sweep(args, torch, jr, wl)}), flush=True)
        return
    if args.leg.startswith("single_4096"):
        dt = args.leg.rsplit("_", 1)[1]
        fr = [wl.single_4096(s, it, dt) for it in (100, 1000) for s in range(4)]
        outs = [torch.empty((f.height, f.width), dtype=torch.int32, device="cuda") for f in fr]
        t0 = time.perf_counter()  # settle the clock, as settle_clocks does
        while time.perf_counter() - t0 < SETTLE_S:
            time_renders(jr, torch, fr, outs, 1, plain=args.plain, schedule=forced)
        time_renders(jr, torch, fr, outs, args.warmup, plain=args.plain, schedule=forced)
        ms = time_renders(jr, torch, fr, outs, args.steps, plain=args.plain, schedule=forced)
        iters = count_sum(torch, outs)
        sched = ("plain" if args.plain else forced.__dict__ if forced is not None
                 else "per-image schedules from the autotune cache")
    else:
        dt = args.leg.rsplit("_", 1)[1]
        fr = wl.parameter_path(dtype=dt)
        sc = jr.Schedule(kernel="plain") if args.plain else forced if forced is not None \
            else tuned_schedule_or_default(jr, args.leg)[0]
        plan = jr.Plan(fr, sc)
        plan.capture()
        settle_clocks(torch, plan)
        ms, _ = time_plan_steps(torch, plan, args.steps, args.warmup, graph=True)
        iters = count_sum(torch, plan.views)
        plan.close()
        sched = sc.__dict__ if sc else "library default"
    print(json.dumps({"leg": args.leg, "plain": args.plain, "ms_per_step": round(ms, 4),
                      "gpixel_iter_s": round(iters / (ms * 1e-3) / 1e9, 2),
                      "pixel_iters": iters, "schedule": sched, "steps": args.steps}),
          flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported: the path has no "
              "exchange between GPUs (several GPUs would each render their own share "
              "of the frames)" % args.gpus, file=sys.stderr)
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
    if args.leg != "headline":
        run_leg(args, torch, jr, wl)
        return
    frames = wl.parameter_path()
    if args.schedule == "plain":
        sched, sched_src = jr.Schedule(kernel="plain"), "--schedule plain"
    elif args.schedule == "tiled":
        sched, sched_src = jr.Schedule(64, 64, 8, 0, 32, 0, 16, "cost"), "--schedule tiled"
    else:
        sched, sched_src = tuned_schedule(jr, "parameter_path_fp32", frames)
    plan = jr.Plan(frames, sched)
    plan.capture()
    settle_ms = settle_clocks(torch, plan)
    ms_step, kernel_ms = time_plan_steps(torch, plan, args.steps, args.warmup, graph=True)
    iters = count_sum(torch, plan.views)
    info = plan.info()
    plan.close()
    pixels = sum(f.pixels for f in frames)
    traffic, traffic_src = measured_traffic(kernel_instance(sched), "parameter_path_fp32",
                                            sched.__dict__)
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
                   "clock_settle_ms": round(settle_ms, 1),
                   "tiles": info["tiles"], "workgroups": info["workgroups"]},
        "roofline": {"bound": "hbm", "achieved": round(store_gbs, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(store_gbs / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "traffic_source": traffic_src,
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
        cb = cpu_baseline(frames, args.cpu_seconds)
        rate_all, n_all, sample_all = cb["all"]
        rate_1, sample_1 = cb["single"]
        line["cpu_baseline"] = {"value": round(rate_all / 1e9, 5), "unit": "Gpixel-iter/s",
                                "cores": n_all, "kind": "oracle", "sample": sample_all,
                                "cpu_model": cb["cpu_model"], "nproc": cb["nproc"],
                                "cpus_allowed": cb["cpus_allowed"],
                                "single_thread": {"value": round(rate_1 / 1e9, 5), "cores": 1,
                                                  "sample": sample_1}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
