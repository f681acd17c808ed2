"""GPU parity of the general maps Z^d + C (d = 3..8) against the oracle.

Every kernel (refill stream, batched plain, rows) must give the oracle's
general-map counts bit for bit in FP64, FP32 and float-float, for Julia and
Mandelbrot frames, mixed with quadratic frames in one launch, and with the
fused colour store.
"""
import numpy as np
import pytest

import oracle
from workloads import Frame

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402

SCHEDS = [
    None,
    jr.Schedule(64, 16, 1, 0, 16, 1, 16, "cost"),
    jr.Schedule(64, 8, 8, 1, 1, 1, 8, "table"),
    jr.Schedule(13, 7, 4, 1, 5, 1, 4, "table"),
    jr.Schedule(8, 8, 8, 0, 32, 0, 16, "cost"),
    jr.Schedule(kernel="plain", order="table"),
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "hybrid", 8),
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 4),
    jr.Schedule(64, 64, 8, 0, 16, 0, 16, "cost", "rows", 48, 32),
    jr.Schedule(37, 5, 4, 0, 32, 1, 8, "table", "rows", 2),
    jr.Schedule(64, 64, 8, 0, 16, 1, 8, "cost", "rows", 4),
]


def ref(f: Frame):
    return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode, f.degree)


def frames_mixed():
    return [
        Frame(complex(0.4, 0.3), (-1.3, 1.3, -1.2, 1.2), 97, 61, 150, "fp32", "julia", 3),
        Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 64, 48, 100, "fp64"),
        Frame(0j, (-1.5, 1.5, -1.5, 1.5), 70, 66, 120, "fp64", "mandelbrot", 4),
        Frame(complex(0.1, 0.75), (-1.2, 1.2, -1.2, 1.2), 45, 33, 200, "ff", "julia", 5),
        Frame(complex(2.05, 0.1), (-1.6, 1.6, -1.6, 1.6), 40, 40, 60, "fp32", "julia", 3),
        Frame(complex(-0.6, 0.0), (-1.3, 1.3, -1.1, 1.1), 33, 129, 80, "fp64", "julia", 8),
        Frame(0j, (-1.4, 1.4, -1.4, 1.4), 50, 40, 90, "ff", "mandelbrot", 3),
    ]


@pytest.mark.parametrize("degree", [3, 4, 5, 8])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
def test_single_image(dtype, degree):
    W, H = (130, 67) if dtype != "ff" else (80, 50)
    c = complex(0.3, 0.5) if degree % 2 else complex(-0.6, 0.2)
    got = jr.render(c, (-1.4, 1.4, -1.2, 1.2), W, H, 120, dtype, degree=degree)
    torch.cuda.synchronize()
    want = oracle.render(c, (-1.4, 1.4, -1.2, 1.2), W, H, 120, dtype, "julia", degree)
    np.testing.assert_array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("sched", range(len(SCHEDS)))
def test_mixed_batch_one_launch(sched):
    frames = frames_mixed()
    offs, total = jr.arena_layout(frames)
    arena = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    _, views = jr.render_batch(frames, SCHEDS[sched], arena=arena, offsets=offs)
    torch.cuda.synchronize()
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(v.cpu().numpy(), ref(f), err_msg=str(f))


def test_colours_of_general_maps():
    frames = frames_mixed()[:4]
    pal_h = np.random.default_rng(21).integers(0, 2 ** 32, size=257, dtype=np.uint64).astype(np.uint32)
    pal = torch.from_numpy(pal_h.view(np.int32).copy()).cuda()
    for sched in (None, jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 4),
                  jr.Schedule(kernel="plain")):
        _, views = jr.render_batch(frames, sched, palette=pal)
        torch.cuda.synchronize()
        for f, v in zip(frames, views):
            np.testing.assert_array_equal(v.cpu().numpy().view(np.uint32),
                                          oracle.colorize(ref(f), pal_h))


def test_degree_two_frames_unchanged_beside_general_ones():
    """A quadratic frame in a launch that also holds general maps keeps the
    quadratic formulations (FP32 with its fused test)."""
    q = Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 96, 64, 100, "fp32")
    g = Frame(complex(0.4, 0.3), (-1.3, 1.3, -1.2, 1.2), 64, 64, 100, "fp32", "julia", 3)
    _, views = jr.render_batch([q, g], jr.Schedule(64, 16, 8, 1, 32, 0, 16, "cost"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(views[0].cpu().numpy(), oracle.render(
        q.c, q.window, q.width, q.height, q.max_iter, "fp32"))
    np.testing.assert_array_equal(views[1].cpu().numpy(), ref(g))


def test_large_general_frame_sampled():
    f = Frame(complex(0.35, 0.42), (-1.4, 1.4, -1.4, 1.4), 2048, 2048, 500, "fp32", "julia", 3)
    out = jr.render(f.c, f.window, f.width, f.height, f.max_iter, "fp32", degree=3)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    ii = rng.integers(0, f.width, 4000).astype(np.int32)
    jj = rng.integers(0, f.height, 4000).astype(np.int32)
    want = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, "fp32",
                                "julia", 3)
    np.testing.assert_array_equal(out.cpu().numpy()[jj, ii], want)
