"""julia_render_batch_noalloc (the allocation-free batch call) against
julia_render_batch: the same frames and schedule must give the same images,
bit for bit, on two calls in a row, the second with a smaller batch (the
fixed device array keeps the first call's table and counters, which the second
must not read).  Calls go through the C ABI via the Python binding."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SENTINEL = -7


def _frames(seed, n, with_general=True):
    """Mixed frames: dtypes, modes, caps, sizes; every 7th a Z^3 + C frame."""
    from workloads import Frame
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        w = int(rng.integers(17, 140))
        h = int(rng.integers(9, 120))
        dt = ("fp32", "fp64", "ff")[k % 3]
        if k % 5 == 4:
            out.append(Frame(0j, (-2.1, 0.7, -1.2, 1.2), w, h, int(rng.integers(20, 300)), dt,
                             "mandelbrot"))
            continue
        r = 0.3 + 0.6 * rng.random()
        th = 2.0 * math.pi * rng.random()
        deg = 3 if (with_general and k % 7 == 6) else 2
        out.append(Frame(complex(r * math.cos(th), r * math.sin(th)), (-1.6, 1.6, -1.4, 1.4),
                         w, h, int(rng.integers(20, 400)), dt, "julia", deg))
    return out


def _gapped_offsets(frames, gap=13):
    offs, total = [], gap
    for f in frames:
        offs.append(total)
        total += f.width * f.height + gap
    return offs, total


def _schedules(jr):
    return {
        "default": None,
        "queues": jr.Schedule(32, 16, 8, 0, 16, 1, 16, "cost", "tiled", 8, 0),
        "rows": jr.Schedule(64, 16, 8, 0, 16, 0, 16, "table", "rows", 8, 32),
        "rows_queues": jr.Schedule(64, 8, 4, 0, 32, 1, 8, "cost", "rows", 6, 0),
        "deferred": jr.Schedule(16, 16, 8, 1, 32, 0, 16, "cost", "tiled", 8, 0),
        "plain": jr.Schedule(kernel="plain"),
    }


def _pair(jr, torch, frames, sched):
    """(noalloc arena, batch arena), both pre-filled with a sentinel."""
    offs, total = _gapped_offsets(frames)
    a = torch.full((total,), SENTINEL, dtype=torch.int32, device="cuda")
    b = torch.full((total,), SENTINEL, dtype=torch.int32, device="cuda")
    jr.render_batch_noalloc(frames, a, sched, offsets=offs)
    jr.render_batch(frames, sched, arena=b, offsets=offs)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), offs


@pytest.mark.parametrize("name", ["default", "queues", "rows", "rows_queues", "deferred",
                                  "plain"])
def test_noalloc_equals_batch_on_two_calls(name):
    import torch
    import paper_1611_03079_amd as jr
    torch.cuda.set_device(0)
    sched = _schedules(jr)[name]
    big = _frames(11, 57)
    small = _frames(12, 6, with_general=False)
    print("noalloc case %s: %d frames then %d" % (name, len(big), len(small)), flush=True)
    for frames in (big, small):
        a, b, offs = _pair(jr, torch, frames, sched)
        assert np.array_equal(a, b), name
        # the frames were written and the gaps between them were not
        gaps = np.ones(a.size, dtype=bool)
        for o, f in zip(offs, frames):
            gaps[o: o + f.width * f.height] = False
        assert (a[gaps] == SENTINEL).all()
        assert (a[~gaps] >= 0).all()


def test_noalloc_single_frame_and_the_largest_batch():
    """One frame (it travels in the kernel arguments; with the queues the
    counters are still the array's) and JR_NOALLOC_MAX_FRAMES small frames."""
    import torch
    import paper_1611_03079_amd as jr
    from workloads import Frame
    torch.cuda.set_device(0)
    one = [Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 300, 200, 150, "fp32")]
    for sched in (None, _schedules(jr)["queues"]):
        print("noalloc single frame, schedule %s" % (sched,), flush=True)
        a, b, _ = _pair(jr, torch, one, sched)
        assert np.array_equal(a, b)
    rng = np.random.default_rng(5)
    many = [Frame(complex(0.7885 * math.cos(t), 0.7885 * math.sin(t)), (-1.6, 1.6, -1.6, 1.6),
                  int(rng.integers(4, 24)), int(rng.integers(4, 24)), 100,
                  ("fp32", "fp64")[k % 2])
            for k, t in enumerate(2.0 * math.pi * rng.random(jr.NOALLOC_MAX_FRAMES))]
    for sched in (None, _schedules(jr)["queues"]):
        print("noalloc %d frames, schedule %s" % (len(many), sched), flush=True)
        a, b, _ = _pair(jr, torch, many, sched)
        assert np.array_equal(a, b)
    # then a smaller batch again: nothing of the large table may leak into it
    few = many[:3]
    a, b, _ = _pair(jr, torch, few, _schedules(jr)["queues"])
    assert np.array_equal(a, b)
