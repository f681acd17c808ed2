"""GPU parity: the HIP kernels against the CPU oracle, element by element.

Every call goes through the C ABI of libjulia.so.  FP64 counts must equal the
oracle's FP64 counts exactly; the FP32 and float-float kernels must equal the
oracle's FP32 and float-float formulations exactly, and their difference from
FP64 is reported as a pixel fraction.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import Frame

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402

UNIT = (-1.5, 1.5, -1.5, 1.5)
C1 = complex(-0.8, 0.156)

# tile_w, tile_h, unroll, defer, refill, persistent, waves_per_cu, order
SCHEDULES = [
    jr.Schedule(64, 16, 1, 0, 16, 1, 16, "cost"),
    jr.Schedule(64, 16, 4, 0, 16, 1, 16, "cost"),
    jr.Schedule(64, 8, 8, 1, 1, 1, 8, "table"),
    jr.Schedule(32, 4, 16, 1, 64, 1, 32, "cost"),
    jr.Schedule(13, 7, 4, 1, 5, 1, 4, "table"),   # ragged tiles, few waves
    jr.Schedule(8, 8, 8, 0, 32, 0, 16, "cost"),   # one wave per tile
    jr.Schedule(64, 64, 2, 0, 48, 0, 16, "table"),
    jr.Schedule(1, 1, 1, 0, 1, 1, 4, "cost"),     # one-pixel tiles
    jr.Schedule(kernel="plain", order="table"),   # one thread per pixel, batched
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "hybrid", 8),
    jr.Schedule(32, 8, 8, 1, 32, 1, 16, "table", "hybrid", 3),
    jr.Schedule(16, 16, 4, 0, 48, 0, 16, "cost", "hybrid", 1),
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 4),   # two phases per tile
    jr.Schedule(37, 5, 4, 0, 32, 1, 8, "table", "rows", 2),   # ragged tiles, work queues
    jr.Schedule(64, 64, 8, 0, 8, 0, 16, "cost", "rows", 1),   # 64-row tiles, one-wave workgroups
    jr.Schedule(1, 1, 4, 0, 1, 1, 4, "cost", "rows", 64),     # one-pixel tiles, long first block
    jr.Schedule(64, 64, 4, 0, 8, 1, 8, "table", "rows", 8),   # several list drains per tile
    jr.Schedule(64, 64, 8, 0, 16, 0, 16, "cost", "rows", 64, 48),  # groups hand off early
    jr.Schedule(37, 5, 4, 0, 32, 1, 8, "table", "rows", 12, 128),  # often after one trip
    # the rows kernel's drain in blocks that test their last iterate
    jr.Schedule(64, 16, 8, 1, 16, 0, 16, "cost", "rows", 4),
    jr.Schedule(64, 64, 4, 1, 8, 1, 8, "table", "rows", 8),     # several drains, queues
    jr.Schedule(64, 32, 8, 1, 16, 0, 16, "table", "rows", 64, 128),
]


def gpu(c, win, W, H, it, dtype, mode="julia", plain=False):
    out = jr.render(c, win, W, H, it, dtype, mode=mode, plain=plain)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def batch(frames, schedule=None, fill=None, offsets=None, rows=None):
    offs, total = jr.arena_layout(frames) if offsets is None else (offsets, None)
    if total is None:
        total = max(o + f.width * f.height for o, f in zip(offs, frames))
    arena = torch.full((total,), -7 if fill is None else fill, dtype=torch.int32, device="cuda")
    arena, views = jr.render_batch(frames, schedule, arena=arena, offsets=offs, rows=rows)
    torch.cuda.synchronize()
    return arena.cpu().numpy(), [v.cpu().numpy() for v in views]


def ref(f: Frame):
    return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode,
                         getattr(f, "degree", 2))


# ------------------------------------------------------------- single images
SHAPES = [(512, 512), (1, 1), (1, 97), (97, 1), (7, 13), (65, 33), (130, 67)]


@pytest.mark.parametrize("plain", [True, False], ids=["plain", "tuned"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s)
def test_fp64_bit_exact(shape, plain):
    W, H = shape
    got = gpu(C1, UNIT, W, H, 100, "fp64", plain=plain)
    np.testing.assert_array_equal(got, oracle.render(C1, UNIT, W, H, 100, "fp64"))


@pytest.mark.parametrize("plain", [True, False], ids=["plain", "tuned"])
@pytest.mark.parametrize("dtype", ["fp32", "ff"])
def test_reduced_precision_matches_formulation(dtype, plain):
    W, H = (512, 512) if dtype == "fp32" else (256, 200)
    got = gpu(C1, UNIT, W, H, 100, dtype, plain=plain)
    np.testing.assert_array_equal(got, oracle.render(C1, UNIT, W, H, 100, dtype))
    frac = float((got != oracle.render(C1, UNIT, W, H, 100, "fp64")).mean())
    assert frac <= 0.005, frac


@pytest.mark.parametrize("plain", [True, False], ids=["plain", "tuned"])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
def test_mandelbrot(dtype, plain):
    win = (-2.2, 0.8, -1.2, 1.3)
    W, H = (300, 250) if dtype != "ff" else (150, 125)
    got = gpu(0j, win, W, H, 200, dtype, mode="mandelbrot", plain=plain)
    np.testing.assert_array_equal(got, oracle.render(0j, win, W, H, 200, dtype, "mandelbrot"))


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_schedules_do_not_change_counts(dtype, sched):
    W, H = (200, 150) if dtype != "ff" else (120, 90)
    f = Frame(complex(-0.4, 0.6), (-1.6, 1.6, -1.2, 1.2), W, H, 300, dtype)
    _, views = batch([f], SCHEDULES[sched])
    np.testing.assert_array_equal(views[0], ref(f))


@pytest.mark.parametrize("c", [complex(-2.0, 0.0), complex(2.5, 0.3), complex(1.95, 0.0),
                               complex(0.25, 0.0), complex(0.0, 1.0)])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
def test_special_constants(c, dtype):
    """|C| > 1.9 runs without deferred tests; C = -2, 1/4, i have exact orbits."""
    win = (-2.1, 2.1, -0.9, 0.9)
    W, H = 81, 41  # odd: the centre row is y = 0 exactly
    for s in (SCHEDULES[1], SCHEDULES[3], SCHEDULES[5]):
        f = Frame(c, win, W, H, 500, dtype)
        _, views = batch([f], s)
        np.testing.assert_array_equal(views[0], ref(f))


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
def test_cap_edge_cases(dtype):
    for it in (0, 1, 2, 3, 5, 17):
        for s in (SCHEDULES[0], SCHEDULES[3], SCHEDULES[6]):
            f = Frame(C1, UNIT, 37, 29, it, dtype)
            _, views = batch([f], s)
            np.testing.assert_array_equal(views[0], ref(f))
    assert not gpu(C1, UNIT, 40, 30, 0, dtype).any()
    assert not gpu(C1, UNIT, 40, 30, 0, dtype, plain=True).any()


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_cap_edge_cases_rows(dtype):
    """Caps around the rows kernel's first-block boundaries (multiples of 4,
    P itself, one either side) with and without early handoff."""
    scheds = [jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 8, 0),
              jr.Schedule(64, 32, 8, 0, 16, 0, 16, "cost", "rows", 48, 96),
              jr.Schedule(64, 64, 4, 0, 8, 0, 16, "cost", "rows", 12, 256)]
    for it in (0, 1, 3, 4, 5, 7, 8, 9, 11, 12, 13, 47, 48, 49, 60):
        f = Frame(C1, UNIT, 70, 37, it, dtype)
        for s in scheds:
            _, views = batch([f], s)
            np.testing.assert_array_equal(views[0], ref(f), err_msg="cap %d %s" % (it, s))


def test_fp64_groups_ending_their_first_trip_early():
    """FP64 row pairs whose pixels have all escaped by the second or third
    test of the first trip end it there.  With C = 0 a pixel's count is
    fixed by |Z0| alone (0 beyond 2, 1 down to 2^(1/2), 2 down to 2^(1/4)),
    so these windows hold whole row pairs of largest count 0, 1 and 2 next
    to pairs that run on; caps straddle the ends (0..5), tiles are ragged,
    and one batch mixes in an FP32 frame (pairs there too, no early end)."""
    frames = [Frame(0j, (0.9, 2.3, -0.3, 0.3), 150, 45, 0, "fp64"),
              Frame(0j, (1.2, 1.4, -0.05, 0.05), 64, 9, 0, "fp64"),
              Frame(0j, (1.45, 1.95, -0.2, 0.2), 70, 8, 0, "fp64"),
              Frame(0j, (2.1, 3.0, -1.0, 1.0), 65, 6, 0, "fp64")]
    # the oracle's largest count over each pair of rows in each 64-column block
    pair_max = set()
    for f in frames:
        img = ref(Frame(f.c, f.window, f.width, f.height, 100, f.dtype))
        for j in range(0, f.height - 1, 2):
            for i in range(0, f.width, 64):
                pair_max.add(int(img[j:j + 2, i:i + 64].max()))
    assert {0, 1, 2} <= pair_max and max(pair_max) > 4, pair_max
    scheds = [jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 4, 0),
              jr.Schedule(64, 8, 4, 0, 16, 0, 16, "table", "rows", 12, 128),
              jr.Schedule(37, 5, 4, 0, 32, 1, 8, "table", "rows", 8, 0)]
    for cap in (0, 1, 2, 3, 4, 5, 100):
        fs = [Frame(f.c, f.window, f.width, f.height, cap, f.dtype) for f in frames]
        fs.append(Frame(0j, (0.9, 2.3, -0.3, 0.3), 97, 11, cap, "fp32"))
        for s in scheds:
            _, views = batch(fs, s)
            for f, v in zip(fs, views):
                np.testing.assert_array_equal(v, ref(f), err_msg="cap %d %s %s" % (cap, f, s))


# ------------------------------------------------------------------ batches
def mixed_frames():
    return [
        Frame(C1, UNIT, 160, 120, 100, "fp64"),
        Frame(complex(0.285, 0.01), (-1.3, 1.1, -0.7, 0.95), 97, 61, 250, "fp32"),
        Frame(0j, (-2.0, 1.0, -1.0, 1.3), 64, 64, 150, "ff", "mandelbrot"),
        Frame(complex(-2.0, 0.0), (-2.1, 2.1, -0.5, 0.5), 31, 9, 64, "fp32"),
        Frame(complex(-0.123, 0.745), (-1.6, 1.6, -1.2, 1.2), 1, 1, 1000, "fp64"),
        Frame(complex(0.3, 0.5), (-1.2, 1.2, -1.2, 1.2), 200, 3, 0, "ff"),
        Frame(0j, (-0.75, -0.74, 0.1, 0.11), 90, 70, 2000, "fp64", "mandelbrot"),
    ]


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_deferred_drain_blocks_at_the_cap(dtype):
    """Deferred drain blocks where the cap falls inside a block (caps 37,
    101, 203 are not multiples of 4 or 8), in Julia and Mandelbrot frames
    (a lane's own C in the replay), in launches of one dtype (which take
    the deferred blocks) and mixed with the other dtype (counted blocks)."""
    for K in (4, 8):
        sched = jr.Schedule(64, 16, K, 1, 16, 0, 16, "cost", "rows", 8)
        for cap in (37, 101, 203):
            frames = [Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 97, 61, cap, dtype),
                      Frame(0j, (-1.3, 0.5, -1.1, 1.1), 80, 70, cap, dtype, "mandelbrot")]
            _, views = batch(frames, sched)
            for f, v in zip(frames, views):
                np.testing.assert_array_equal(v, ref(f), err_msg="%s K=%d cap=%d" % (f, K, cap))
            other = "fp64" if dtype == "fp32" else "fp32"
            mixed = frames + [Frame(complex(0.285, 0.01), (-1.2, 1.2, -0.9, 0.9), 50, 40, cap,
                                    other)]
            _, views = batch(mixed, sched)
            for f, v in zip(mixed, views):
                np.testing.assert_array_equal(v, ref(f), err_msg="mixed %s" % (f,))


@pytest.mark.parametrize("sched", [None, *range(len(SCHEDULES))])
def test_mixed_batch_one_launch(sched):
    frames = mixed_frames()
    # gaps between frames stay untouched (sentinel -7): no stray or lost tile
    offs, pos = [], 5
    for f in frames:
        offs.append(pos)
        pos += f.pixels + 3
    arena, views = batch(frames, None if sched is None else SCHEDULES[sched], offsets=offs)
    covered = np.zeros(arena.size, dtype=bool)
    for o, f, v in zip(offs, frames, views):
        np.testing.assert_array_equal(v, ref(f))
        covered[o:o + f.pixels] = True
    assert (arena[~covered] == -7).all()


@pytest.mark.parametrize("sched", [jr.Schedule(4, 4, 4, 0, 16, 1, 4, "table"),
                                   jr.Schedule(8, 2, 8, 1, 8, 1, 4, "table"),
                                   jr.Schedule(3, 5, 2, 0, 64, 0, 16, "table"),
                                   jr.Schedule(kernel="plain", order="table"),
                                   jr.Schedule(5, 3, 8, 1, 16, 1, 4, "table", "hybrid", 2),
                                   jr.Schedule(8, 8, 2, 0, 8, 0, 16, "table", "hybrid", 5)])
def test_variant_switches_inside_a_wave(sched):
    """Frames alternate dtype, mode and absorbing/non-absorbing C in table order
    with small tiles, so a wave's stream changes variant many times."""
    cs = [complex(-0.8, 0.156), complex(2.2, 0.1), complex(0.3, -0.5), complex(-1.95, 0.05)]
    frames = []
    for k in range(36):
        dt = ("fp64", "fp32", "ff")[k % 3]
        mode = "mandelbrot" if k % 5 == 4 else "julia"
        win = (-2.1, 1.0, -1.2, 1.1) if mode == "mandelbrot" else (-1.7, 1.6, -1.3, 1.2)
        frames.append(Frame(cs[k % 4], win, 23 + k, 17 + (k % 7), 40 + 13 * k, dt, mode))
    _, views = batch(frames, sched)
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(v, ref(f))


def test_batch_equals_single_renders():
    frames = [Frame(c, UNIT, 120, 90, 100, dt) for c in (C1, complex(0.3, 0.02), complex(-1.0, 0.25))
              for dt in ("fp64", "fp32", "ff")]
    _, views = batch(frames)
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(v, gpu(f.c, f.window, f.width, f.height, f.max_iter, f.dtype))


def test_row_ranges():
    f = Frame(C1, UNIT, 70, 50, 100, "fp32")
    full = ref(f)
    _, views = batch([f], SCHEDULES[1], rows=[(13, 31)])
    v = views[0]
    np.testing.assert_array_equal(v[13:31], full[13:31])
    assert (v[:13] == -7).all() and (v[31:] == -7).all()


def test_plan_launch_and_graph_replay():
    frames = wl.parameter_path(n=8, width=240, height=135)
    plan = jr.Plan(frames, jr.Schedule(64, 16, 4, 0, 16, 1, 16, "cost"))
    want = [oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype) for f in frames]
    plan.arena.fill_(-1)
    plan.launch()
    torch.cuda.synchronize()
    for v, w in zip(plan.views, want):
        np.testing.assert_array_equal(v.cpu().numpy(), w)
    plan.capture()
    for rep in range(4):
        plan.arena.fill_(-1)          # eager work between the replays
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        for v, w in zip(plan.views, want):
            np.testing.assert_array_equal(v.cpu().numpy(), w)
    plan.close()


def test_single_frame_render_in_torch_graph():
    """A one-frame render carries its frame in the kernel arguments, so a torch
    CUDA graph can capture it; every replay (with eager work between) gives
    the oracle's counts."""
    f = Frame(C1, UNIT, 300, 200, 150, "fp32")
    out = torch.empty((200, 300), dtype=torch.int32, device="cuda")
    jr.render(f.c, f.window, 300, 200, 150, "fp32", out=out)   # warm up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        jr.render(f.c, f.window, 300, 200, 150, "fp32", out=out,
                  schedule=jr.Schedule(64, 16, 8, 0, 32, 0, 16, "cost"))
    want = ref(f)
    for _ in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)


def test_streams_are_independent():
    f1 = Frame(C1, UNIT, 256, 256, 300, "fp64")
    f2 = Frame(complex(0.3, 0.5), UNIT, 256, 256, 300, "fp32")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            a, va = jr.render_batch([f1], stream=s1)
        with torch.cuda.stream(s2):
            b, vb = jr.render_batch([f2], stream=s2)
        outs.append((a, va, b, vb))
    torch.cuda.synchronize()
    for a, va, b, vb in outs:
        np.testing.assert_array_equal(va[0].cpu().numpy(), ref(f1))
        np.testing.assert_array_equal(vb[0].cpu().numpy(), ref(f2))


# ------------------------------------------------------------ full sizes
def _sample(W, H, n, seed):
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, W, n).astype(np.int32)
    jj = rng.integers(0, H, n).astype(np.int32)
    # always include the corners and the centre
    ii = np.concatenate([ii, [0, W - 1, 0, W - 1, W // 2]]).astype(np.int32)
    jj = np.concatenate([jj, [0, 0, H - 1, H - 1, H // 2]]).astype(np.int32)
    return ii, jj


def oracle_images(frames):
    """The oracle's whole images of `frames`, rendered by a pool of host
    threads (the oracle library releases the interpreter lock while it runs,
    so each frame is one single-threaded oracle call on its own core)."""
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as pool:
        return list(pool.map(ref, frames))


def _first_difference(got, want):
    bad = np.argwhere(got != want)
    j, i = bad[0]
    return "%d pixels differ; first at row %d column %d: %d != %d" % (
        len(bad), j, i, got[j, i], want[j, i])


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_single_4096_whole_images(dtype):
    """The 4096 x 4096 single images (C = 0.7885 e^{i theta}, seeds 0..3,
    caps 100 and 1000) in the tuned and the plain kernel, each compared
    whole with the oracle's image."""
    frames = [wl.single_4096(seed, it, dtype) for it in (100, 1000) for seed in range(4)]
    want = oracle_images(frames)
    for f, w in zip(frames, want):
        for plain in (False, True):
            got = gpu(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, plain=plain)
            if not np.array_equal(got, w):
                raise AssertionError("%s plain=%s: %s" % (f, plain, _first_difference(got, w)))


def _golden_rows(name):
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        if not line.startswith("#"):
            rows.append(line.split()[1:])
    return rows


def _digest(view):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(view.cpu().numpy(), dtype="<i4").tobytes()).hexdigest()


def _bench_schedule(name):
    from paper_1611_03079_amd import autotune as at
    e = at.load_cache().get("_workloads", {}).get(name)
    return jr.Schedule(**e["schedule"]) if e else None


@pytest.mark.parametrize("workload", ["parameter_path_fp32", "general_deg3_fp32"])
def test_full_batch_whole_images(workload):
    """The benchmark's batches at full size, in its launch setup (autotuned
    schedule, captured graph replayed): every frame's whole image against
    the oracle's, through the SHA-256 digests of the oracle's images
    (tests/golden, written by the oracle).  A frame whose digest differs is
    rendered by the oracle here and the differing pixels are reported."""
    if workload == "parameter_path_fp32":
        frames, golden = wl.parameter_path(), "parameter_path_fp32_digests.txt"
    else:
        frames, golden = wl.general_path(32, 3), "general_path_deg3_fp32_digests.txt"
    want = _golden_rows(golden)
    assert len(want) == len(frames)
    plan = jr.Plan(frames, _bench_schedule(workload))
    plan.arena.fill_(-1)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    bad = []
    for k, (f, v, (d, s)) in enumerate(zip(frames, plan.views, want)):
        if _digest(v) != d:
            got = v.cpu().numpy()
            bad.append("frame %d: %s" % (k, _first_difference(got, ref(f))))
        assert int(v.sum(dtype=torch.int64)) == int(s) or bad
    plan.close()
    assert not bad, "; ".join(bad[:5])


def test_uneven_batch_whole_fp32_frames_sampled_ff():
    """The 1024-frame uneven batch (sides 256..4096, caps 100/500/2000, FP32
    and float-float, 24.5 GB of counts) in one launch with the benchmark's
    schedule.  Every FP32 frame whole against the digest of the oracle's
    image (tests/golden/uneven_batch_fp32_digests.txt, written by the
    oracle); every float-float frame (the oracle's float-float arithmetic
    would take a day for them all) on 512 sampled pixels, and every 8th
    also on a whole row through its middle."""
    from concurrent.futures import ThreadPoolExecutor
    frames = wl.uneven_batch(0, n=1024)
    want = {int(k): (d, int(sm)) for k, d, sm in
            (l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden",
                                                   "uneven_batch_fp32_digests.txt"))
             if not l.startswith("#"))}
    assert sorted(want) == [k for k, f in enumerate(frames) if f.dtype == "fp32"]
    arena, views = jr.render_batch(frames, _bench_schedule("uneven_fp32_ff"))
    torch.cuda.synchronize()
    bad = [k for k, (d, _) in want.items() if _digest(views[k]) != d]
    if bad:
        k = bad[0]
        detail = _first_difference(views[k].cpu().numpy(), ref(frames[k]))
        raise AssertionError("%d FP32 frames differ; frame %d (%s): %s" % (
            len(bad), k, frames[k], detail))
    rng = np.random.default_rng(17)
    jobs = []
    for k, f in enumerate(frames):
        if f.dtype != "ff":
            continue
        ii = rng.integers(0, f.width, 512).astype(np.int32)
        jj = rng.integers(0, f.height, 512).astype(np.int32)
        if len(jobs) % 8 == 0:
            ii = np.concatenate([ii, np.arange(f.width, dtype=np.int32)])
            jj = np.concatenate([jj, np.full(f.width, f.height // 2, dtype=np.int32)])
        got = views[k][torch.from_numpy(jj).long().cuda(),
                       torch.from_numpy(ii).long().cuda()].cpu().numpy()
        jobs.append((f, ii, jj, got))

    def check(job):
        f, ii, jj, got = job
        w = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        return None if np.array_equal(got, w) else "%s: %d of %d sampled pixels differ" % (
            f, int((got != w).sum()), got.size)

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as pool:
        errs = [e for e in pool.map(check, jobs) if e]
    assert len(jobs) == 1024 - len(want) and not errs, errs[:3]
    del arena, views
    torch.cuda.empty_cache()


def test_largest_frame():
    """A frame of 2^31 - 1 - 2^16 pixels (the limit is < 2^31): counts 0 outside
    the escape radius, and a band through the set checked against the oracle."""
    W = 65535
    H = (2 ** 31 - 1 - 2 ** 16) // W
    win = (-2.0, 2.0, -1.5, 1.5)
    out = torch.empty((H, W), dtype=torch.int32, device="cuda")
    jr.render(complex(-0.8, 0.156), win, W, H, 20, "fp32", out=out)
    torch.cuda.synchronize()
    ii, jj = _sample(W, H, 5000, 11)
    got = out[torch.from_numpy(jj).long().cuda(), torch.from_numpy(ii).long().cuda()].cpu().numpy()
    want = oracle.render_pixels(complex(-0.8, 0.156), win, W, H, 20, ii, jj, "fp32")
    np.testing.assert_array_equal(got, want)
    del out
    torch.cuda.empty_cache()


# ------------------------------------------------ paths and zooms (Section 3)
def test_cardioid_path_batch():
    """The prescribed path of Section 3: C on f(t) with a = 3.9, then a growing
    cardioid (a = 3.7), as one batched launch."""
    frames = (wl.cardioid_path(12, 3.9, width=200, height=112, max_iter=200)
              + wl.cardioid_path(6, 3.7, width=160, height=90, max_iter=150, dtype="fp64"))
    _, views = batch(frames)
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(v, ref(f))


@pytest.mark.parametrize("width", [1e-3, 1e-5, 1e-7])
def test_deep_zoom_windows(width):
    """Narrow windows on the Mandelbrot set (C from Figure 3's deep zoom) and on
    a Julia set: FP64 exact, float-float exact to its formulation, and its
    difference from FP64 reported."""
    cx, cy = 0.177078, 0.577384
    win = (cx - width / 2, cx + width / 2, cy - width / 2, cy + width / 2)
    for mode in ("mandelbrot", "julia"):
        c = complex(cx, cy) if mode == "julia" else 0j
        fr = [Frame(c, win, 96, 96, 600, dt, mode) for dt in ("fp64", "ff")]
        _, views = batch(fr)
        for f, v in zip(fr, views):
            np.testing.assert_array_equal(v, ref(f))


def test_rows_wide_frame_offsets():
    """A frame 2^25 pixels wide and 40 rows tall: pixels of rows 32 and below
    lie more than 2^32 bytes past their tile's first pixel.  The rows kernel
    writes them from its list drain; sampled survivors of those rows against
    the oracle (a 32-bit byte offset would have wrapped onto other pixels)."""
    W, H = 1 << 25, 40
    win = (-1.6, 1.6, -0.05, 0.05)
    c, cap = complex(-0.4, 0.6), 48
    sched = jr.Schedule(64, 64, 8, 0, 16, 0, 16, "cost", "rows", 8)
    out = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    jr.render(c, win, W, H, cap, "fp32", out=out, schedule=sched)
    torch.cuda.synchronize()
    rng = np.random.default_rng(23)
    jj = rng.integers(32, H, 4000).astype(np.int32)
    ii = rng.integers(0, W, 4000).astype(np.int32)
    want = oracle.render_pixels(c, win, W, H, cap, ii, jj, "fp32")
    # the samples must include pixels that outlive the first block (P = 8)
    assert (want > 8).sum() >= 100
    got = out[torch.from_numpy(jj).long().cuda(), torch.from_numpy(ii).long().cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, want)
    del out
    torch.cuda.empty_cache()


def test_plan_info_reports_the_launched_grid():
    """jr_plan_info counts the workgroups actually launched: one per tile for
    dispatched rows tiles (counts, or colours from a small FP32 palette), one
    per four tiles otherwise."""
    frames = [Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 200, 130, 100, "fp32")]
    rows = jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 16, 32)
    tiled = jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost")
    small = torch.arange(100, dtype=torch.int32, device="cuda")
    large = torch.arange(300, dtype=torch.int32, device="cuda")
    for sched, pal, one_per_tile in ((rows, None, True), (rows, small, True),
                                     (rows, large, False), (tiled, None, False)):
        plan = jr.Plan(frames, sched)
        try:
            if pal is not None:
                plan.set_palette(pal)
            info = plan.info()
            want = info["tiles"] if one_per_tile else (info["tiles"] + 3) // 4
            assert info["tiles"] == 4 * 9 and info["workgroups"] == want, (sched, info)
            plan.launch()
            torch.cuda.synchronize()
        finally:
            plan.close()


def test_point_symmetry_of_the_full_parameter_path():
    """Z -> -Z maps every orbit of Z^2 + C onto one with the same |Z|, and the
    three formulations commute with that sign change exactly (squares and the
    (2x)y product see both signs flipped; round-to-nearest is odd).  On a
    window centred on 0 the binary64 pixel centres of (i, j) and
    (W-1-i, H-1-j) are exact negatives, so every image equals itself turned
    by 180 degrees.  Checked on all 256 frames at full size (530 M pixels)
    with the tuned schedule of the benchmark, and on FP64 and float-float
    frames of the path."""
    from paper_1611_03079_amd import autotune as at
    frames = wl.parameter_path()
    e = at.load_cache().get("_workloads", {}).get("parameter_path_fp32")
    sched = jr.Schedule(**e["schedule"]) if e else None
    arena, views = jr.render_batch(frames, sched)
    for k, v in enumerate(views):
        assert torch.equal(v, v.flip(0).flip(1)), "frame %d" % k
    del arena, views
    others = [Frame(f.c, f.window, 640, 360, f.max_iter, dt)
              for f in frames[::37] for dt in ("fp64", "ff")]
    _, views = batch(others, None)
    for f, v in zip(others, views):
        assert (v == v[::-1, ::-1]).all(), str(f)
    torch.cuda.empty_cache()


def test_mirror_symmetry_of_mandelbrot_frames():
    """With Z_0 = 0 the orbit of conj(C) is the conjugate orbit, and the
    formulations commute with conjugation exactly; on a window symmetric in
    Im the image equals its top-bottom mirror."""
    frames = [Frame(0j, (-2.1, 0.7, -1.2, 1.2), 700, 601, 300, dt, "mandelbrot")
              for dt in ("fp64", "fp32", "ff")]
    for sched in (None, jr.Schedule(64, 32, 8, 0, 16, 0, 16, "cost", "rows", 48, 96)):
        _, views = batch(frames, sched)
        for f, v in zip(frames, views):
            assert (v == v[::-1, :]).all(), str(f)
