"""The prescribed cardioid path of Section 3 with its constants generated on
the device (julia_render_cardioid_path, jr_plan_create_cardioid): every frame
equals the oracle's image for the oracle's own constant of that frame
(jro_cardioid_constant, the same definition implemented separately), so the
generator and the renderer are checked together, bit for bit."""
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import Frame

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402


def as_path(g):
    return jr.CardioidPath(g.step, g.a0, g.da, g.window, g.frames, g.width, g.height,
                           g.max_iter, g.dtype)


def oracle_frames(g):
    return [Frame(oracle.cardioid_constant(g.step, g.a0, g.da, k), g.window, g.width, g.height,
                  g.max_iter, g.dtype) for k in range(g.frames)]


def ref(f):
    return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype)


SCHEDS = [None,
          jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 16, 32),
          jr.Schedule(16, 16, 8, 1, 32, 0, 16, "cost"),
          jr.Schedule(32, 8, 4, 0, 16, 1, 8, "table"),
          jr.Schedule(kernel="plain")]


@pytest.mark.parametrize("sched", range(len(SCHEDS)))
@pytest.mark.parametrize("dtype", ["fp32", "fp64", "ff"])
def test_small_path_one_call(dtype, sched):
    """Three trips of 16 frames while a shrinks from 3.9 to 3.3 (the cardioid
    grows), 161 x 91 pixels: every frame whole against the oracle."""
    g = wl.growing_cardioid_path(48, 16, 3.9, 3.3, 161, 91, 150, dtype)
    _, views = jr.render_cardioid_path(as_path(g), SCHEDS[sched])
    torch.cuda.synchronize()
    for k, f in enumerate(oracle_frames(g)):
        np.testing.assert_array_equal(views[k].cpu().numpy(), ref(f), err_msg="frame %d" % k)


def test_plan_replays_generate_the_same_frames():
    """A plan generates its table on the device at every launch: a captured
    graph replayed several times, with other work between the replays, gives
    the oracle's images every time."""
    g = wl.growing_cardioid_path(24, 12, 3.9, 3.6, 120, 70, 120, "fp32")
    want = [ref(f) for f in oracle_frames(g)]
    plan = jr.Plan.cardioid(as_path(g), jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 8))
    plan.capture()
    for rep in range(3):
        plan.arena.fill_(-1)
        plan.replay()
        torch.cuda.synchronize()
        for k, v in enumerate(plan.views):
            np.testing.assert_array_equal(v.cpu().numpy(), want[k], err_msg="replay %d" % rep)
        jr.render(complex(0.3, 0.5), (-1.5, 1.5, -1.5, 1.5), 64, 64, 50, "fp64")
    plan.close()


def test_full_size_path_in_the_bench_launch():
    """The benchmark's path: 256 frames of 1920 x 1080, four trips of 64
    frames while a goes from 3.9 to 3.5, FP32, cap 100, in a captured graph
    with the cardioid schedule of the autotune cache.  Every 16th frame whole
    against the oracle; every frame on 2000 sampled pixels."""
    from concurrent.futures import ThreadPoolExecutor
    from paper_1611_03079_amd import autotune as at
    g = wl.growing_cardioid_path()
    e = at.load_cache().get("_workloads", {}).get("cardioid_path_fp32")
    plan = jr.Plan.cardioid(as_path(g), jr.Schedule(**e["schedule"]) if e else None)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    frames = oracle_frames(g)
    rng = np.random.default_rng(3)

    def check(k):
        f = frames[k]
        got = plan.views[k].cpu().numpy()
        if k % 16 == 0:
            return None if np.array_equal(got, ref(f)) else "frame %d differs" % k
        ii = rng.integers(0, f.width, 2000).astype(np.int32)
        jj = rng.integers(0, f.height, 2000).astype(np.int32)
        w = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        return None if np.array_equal(got[jj, ii], w) else "frame %d: samples differ" % k

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as pool:
        errs = [e for e in pool.map(check, range(g.frames)) if e]
    plan.close()
    assert not errs, errs[:3]
