"""Progress of a plan's launches (jr_plan_set_progress): per-frame done
counters and a stop flag, the bookkeeping that lets a long batch of frames
(Section 3's paths and zooms) stop early and re-render only the frames it
left incomplete.

The images are checked against the oracle; the counters against the frames'
pixel counts.  A stop flag never makes a kernel wait: waves read it before
claiming a tile and exit when it is set, so every launch here ends normally
whether the flag is set before the launch, during it, or never."""
import time

import numpy as np
import pytest

import oracle
from workloads import Frame

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402

ROWS = jr.Schedule(32, 16, 8, 0, 16, 0, 16, "cost", "rows", 16, 32)
ROWS_QUEUES = jr.Schedule(64, 8, 8, 0, 16, 1, 16, "table", "rows", 8, 0)
PLAIN = jr.Schedule(kernel="plain")
TILED = jr.Schedule(16, 16, 8, 1, 32, 0, 16, "cost")
SCHEDS = {"rows": ROWS, "rows_queues": ROWS_QUEUES, "plain": PLAIN}


def mixed_frames():
    """Odd sizes, every dtype, both modes, a cubic map and a rational one."""
    w = (-1.6, 1.6, -1.2, 1.2)
    return [Frame(complex(-0.8, 0.156), w, 97, 61, 150, "fp32"),
            Frame(complex(0.285, 0.01), w, 130, 33, 400, "fp64"),
            Frame(complex(-0.4, 0.6), w, 64, 64, 200, "ff"),
            Frame(0j, (-2.2, 0.8, -1.2, 1.2), 81, 57, 300, "fp64", "mandelbrot"),
            Frame(complex(0.4, 0.3), w, 45, 70, 120, "fp32", degree=3),
            Frame(complex(-0.55, 0.1), w, 77, 49, 100, "fp64", lam=complex(-0.02, 0.01)),
            Frame(complex(-0.7269, 0.1889), w, 1, 1, 50, "fp32"),
            Frame(complex(-0.1, 0.65), w, 200, 3, 500, "fp32")]


def oracle_image(f):
    if f.lam is not None:
        return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype,
                             degree=f.degree, lam=f.lam)
    return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode, f.degree)


def check_images(plan, want, frames=None):
    for k in (range(len(want)) if frames is None else frames):
        np.testing.assert_array_equal(plan.views[k].cpu().numpy(), want[k], err_msg="frame %d" % k)


@pytest.mark.parametrize("sched", sorted(SCHEDS))
def test_counters_reach_every_frame_size(sched):
    """Without a stop, every counter ends at its frame's pixel count, and the
    images equal the oracle's: counting changes no pixel."""
    frames = mixed_frames()
    want = [oracle_image(f) for f in frames]
    plan = jr.Plan(frames, SCHEDS[sched])
    done = torch.full((len(frames),), -5, dtype=torch.int32, device="cuda")
    plan.set_progress(done)
    plan.launch()
    torch.cuda.synchronize()
    assert done.cpu().tolist() == [f.pixels for f in frames]
    assert plan.incomplete(done.cpu()) == []
    check_images(plan, want)
    plan.close()


def test_counters_in_a_replayed_graph():
    """The counters are zeroed by a kernel inside the captured graph: each
    replay, after the host has spoilt them, ends at the pixel counts again."""
    frames = mixed_frames()
    want = [oracle_image(f) for f in frames]
    plan = jr.Plan(frames, ROWS)
    done = torch.zeros(len(frames), dtype=torch.int32, device="cuda")
    plan.set_progress(done)
    plan.capture()
    for rep in range(3):
        done.fill_(1000 + rep)
        plan.arena.fill_(-1)
        plan.replay()
        torch.cuda.synchronize()
        assert done.cpu().tolist() == [f.pixels for f in frames], "replay %d" % rep
        check_images(plan, want)
        jr.render(complex(0.3, 0.5), (-1.5, 1.5, -1.5, 1.5), 64, 64, 50, "fp64")
    plan.close()


@pytest.mark.parametrize("sched", sorted(SCHEDS))
def test_stop_before_the_launch_then_resume(sched):
    """A flag set before the launch: no tile is claimed, every counter stays
    0 and the arena keeps its sentinel.  Cleared, a plan of the incomplete
    frames at their own offsets completes the arena."""
    frames = mixed_frames()
    want = [oracle_image(f) for f in frames]
    plan = jr.Plan(frames, SCHEDS[sched])
    done = torch.zeros(len(frames), dtype=torch.int32, device="cuda")
    stop = torch.ones(1, dtype=torch.int32, device="cuda")
    plan.arena.fill_(-7)
    plan.set_progress(done, stop)
    plan.launch()
    torch.cuda.synchronize()
    assert done.cpu().tolist() == [0] * len(frames)
    assert (plan.arena == -7).all().item()
    todo = plan.incomplete(done.cpu())
    assert todo == list(range(len(frames)))
    stop.zero_()
    rest = jr.Plan([frames[k] for k in todo], SCHEDS[sched], arena=plan.arena,
                   offsets=[plan.offsets[k] for k in todo])
    rest.launch()
    torch.cuda.synchronize()
    check_images(plan, want)
    rest.close()
    plan.close()


def test_progress_needs_the_rows_or_plain_kernel():
    frames = mixed_frames()[:2]
    plan = jr.Plan(frames, TILED)
    done = torch.zeros(len(frames), dtype=torch.int32, device="cuda")
    with pytest.raises(jr.JuliaError, match="rows or plain"):
        plan.set_progress(done)
    plan.close()
    plan = jr.Plan(frames, ROWS)
    with pytest.raises(jr.JuliaError, match="needs done"):
        jr._check(jr.lib.jr_plan_set_progress(plan._h, None, jr.ctypes.c_void_p(done.data_ptr())))
    plan.set_progress(None)  # off again
    plan.launch()
    torch.cuda.synchronize()
    plan.close()


def deep_frames(n, side, cap):
    """Slow frames: windows of width 0.02 on the boundary of the Julia set of
    C = -0.8 + 0.156i, FP64, where many orbits run to the cap."""
    out = []
    for k in range(n):
        cx = -0.6 + 0.01 * (k % 8)
        cy = 0.1 + 0.01 * (k // 8)
        out.append(Frame(complex(-0.8, 0.156), (cx - 0.01, cx + 0.01, cy - 0.01, cy + 0.01),
                         side, side, cap, "fp64"))
    return out


@pytest.mark.parametrize("sched", ["rows", "rows_queues"])
def test_stop_while_running_then_resume(sched):
    """The host sets a pinned flag a few milliseconds into a long launch.
    Frames whose counter reached their pixel count equal the oracle on
    sampled pixels; a second plan over the incomplete frames, at their own
    offsets, completes the batch, after which every frame's samples equal
    the oracle's.  The launch may also finish before the flag is seen: the
    checks hold either way, and the test reports which happened."""
    frames = deep_frames(32, 768, 4000)
    plan = jr.Plan(frames, SCHEDS[sched])
    done = torch.zeros(len(frames), dtype=torch.int32, device="cuda")
    stop = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    plan.arena.fill_(-3)
    plan.set_progress(done, stop)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.launch()
    time.sleep(0.003)
    stop.numpy()[0] = 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = done.cpu().tolist()
    todo = plan.incomplete(d)
    print("stopped after %.1f ms: %d of %d frames incomplete, %d of %d pixels done"
          % (1e3 * (t1 - t0), len(todo), len(frames), sum(d), sum(f.pixels for f in frames)))
    # counters only ever count whole stored tiles, never more than the frame
    assert all(0 <= v <= f.pixels for v, f in zip(d, frames))
    rng = np.random.default_rng(11)
    side = frames[0].width
    ii = rng.integers(0, side, 3000).astype(np.int32)
    jj = rng.integers(0, side, 3000).astype(np.int32)

    def samples_ok(k):
        f = frames[k]
        got = plan.views[k].cpu().numpy()[jj, ii]
        want = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        np.testing.assert_array_equal(got, want, err_msg="frame %d" % k)

    for k in range(len(frames)):
        if k not in todo:
            samples_ok(k)
    stop.numpy()[0] = 0
    if todo:
        rest = jr.Plan([frames[k] for k in todo], SCHEDS[sched], arena=plan.arena,
                       offsets=[plan.offsets[k] for k in todo])
        rest.launch()
        torch.cuda.synchronize()
        rest.close()
    assert not (plan.arena == -3).any().item()
    for k in range(0, len(frames), 3):
        samples_ok(k)
    plan.close()


def test_counters_of_a_cardioid_plan_and_a_colour_store():
    """A plan whose table is generated on the device counts its frames in
    path order; a plan storing colours counts through the colour variant of
    the progress kernels, and its colours equal the oracle's."""
    import workloads as wl
    g = wl.growing_cardioid_path(24, 12, 3.9, 3.6, 120, 70, 120, "fp32")
    path = jr.CardioidPath(g.step, g.a0, g.da, g.window, g.frames, g.width, g.height,
                           g.max_iter, g.dtype)
    plan = jr.Plan.cardioid(path, ROWS)
    done = torch.zeros(g.frames, dtype=torch.int32, device="cuda")
    plan.set_progress(done)
    plan.launch()
    torch.cuda.synchronize()
    assert done.cpu().tolist() == [g.width * g.height] * g.frames
    for k in (0, 7, g.frames - 1):
        f = Frame(oracle.cardioid_constant(g.step, g.a0, g.da, k), g.window, g.width, g.height,
                  g.max_iter, g.dtype)
        np.testing.assert_array_equal(plan.views[k].cpu().numpy(), oracle_image(f))
    plan.close()
    frames = mixed_frames()
    palette = (np.arange(300, dtype=np.uint64) * 2654435761 % 2 ** 32).astype(np.uint32)
    for sched in (ROWS, PLAIN):
        plan = jr.Plan(frames, sched)
        plan.set_palette(torch.from_numpy(palette.view(np.int32).copy()).cuda())
        done = torch.zeros(len(frames), dtype=torch.int32, device="cuda")
        plan.set_progress(done)
        plan.launch()
        torch.cuda.synchronize()
        assert done.cpu().tolist() == [f.pixels for f in frames]
        for k, f in enumerate(frames):
            want = oracle.colorize(oracle_image(f), palette)
            got = plan.views[k].cpu().numpy().view(np.uint32)
            np.testing.assert_array_equal(got, want, err_msg="frame %d" % k)
        plan.close()
