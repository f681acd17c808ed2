"""GPU parity of the fused count -> colour store against the oracle.

The kernels store palette[min(count, len - 1)] in place of the count
(julia_render_batch_colored, julia_render_colored, jr_plan_set_palette).  The
expected image is the oracle's counts coloured by the oracle's table lookup;
every comparison is bit for bit on the 32-bit words.
"""
import numpy as np
import pytest

import oracle
from workloads import Frame

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402

UNIT = (-1.5, 1.5, -1.5, 1.5)
C1 = complex(-0.8, 0.156)


def palette(n, seed=3):
    """Seeded random 32-bit colours (host array, device tensor)."""
    host = np.random.default_rng(seed).integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    return host, torch.from_numpy(host.view(np.int32).copy()).cuda()


def expected(f: Frame, pal_host):
    counts = oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode)
    return oracle.colorize(counts, pal_host)


def as_u32(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


SCHEDS = [
    None,
    jr.Schedule(64, 16, 1, 0, 16, 1, 16, "cost"),
    jr.Schedule(64, 8, 8, 1, 1, 1, 8, "table"),
    jr.Schedule(13, 7, 4, 1, 5, 1, 4, "table"),
    jr.Schedule(8, 8, 8, 0, 32, 0, 16, "cost"),
    jr.Schedule(kernel="plain", order="table"),
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "hybrid", 8),
    jr.Schedule(32, 8, 8, 1, 32, 1, 16, "table", "hybrid", 3),
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 4),
    jr.Schedule(64, 32, 8, 0, 16, 0, 16, "cost", "rows", 32, 32),
]


@pytest.mark.parametrize("plen", [101, 17, 1, 8192])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "ff"])
def test_single_image_colours(dtype, plen):
    W, H = (130, 67)
    ph, pd = palette(plen)
    got = as_u32(jr.render(C1, UNIT, W, H, 100, dtype, palette=pd))
    np.testing.assert_array_equal(got, expected(Frame(C1, UNIT, W, H, 100, dtype), ph))


def test_plain_and_mandelbrot_colours():
    ph, pd = palette(64, seed=5)
    got = as_u32(jr.render(C1, UNIT, 97, 61, 100, "fp64", plain=True, palette=pd))
    np.testing.assert_array_equal(got, expected(Frame(C1, UNIT, 97, 61, 100, "fp64"), ph))
    win = (-2.0, 0.7, -1.2, 1.2)
    got = as_u32(jr.render(0j, win, 90, 80, 200, "fp32", mode="mandelbrot", palette=pd))
    np.testing.assert_array_equal(got, expected(Frame(0j, win, 90, 80, 200, "fp32", "mandelbrot"),
                                                ph))


def test_julia_render_colored_entry_point():
    """The one-image C entry point, called directly."""
    import ctypes
    ph, pd = palette(101, seed=9)
    out = torch.empty((75, 81), dtype=torch.int32, device="cuda")
    rc = jr.lib.julia_render_colored(jr.jr_complex(C1.real, C1.imag), jr._window(UNIT), 81, 75,
                                     100, jr.DTYPES["fp32"], ctypes.c_void_p(pd.data_ptr()), 101,
                                     ctypes.c_void_p(out.data_ptr()), None)
    assert rc == jr.JR_OK, jr.last_error()
    np.testing.assert_array_equal(as_u32(out), expected(Frame(C1, UNIT, 81, 75, 100, "fp32"), ph))


@pytest.mark.parametrize("sched", range(len(SCHEDS)))
def test_mixed_batch_colours(sched):
    frames = [Frame(C1, UNIT, 130, 67, 100, "fp64"),
              Frame(complex(0.285, 0.01), (-1.2, 1.2, -0.9, 0.9), 97, 45, 300, "fp32"),
              Frame(0j, (-2.0, 0.6, -1.1, 1.1), 64, 50, 150, "ff", "mandelbrot"),
              Frame(complex(-0.4, 0.6), (-1.6, 1.6, -1.6, 1.6), 33, 129, 60, "fp32")]
    ph, pd = palette(301, seed=11)
    offs, total = jr.arena_layout(frames)
    arena = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    _, views = jr.render_batch(frames, SCHEDS[sched], arena=arena, offsets=offs, palette=pd)
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(as_u32(v), expected(f, ph))


def test_colours_equal_palette_of_gpu_counts():
    """Same launch configuration with and without the table: the coloured
    image is the table looked up at the counted image (GPU against GPU)."""
    frames = [Frame(complex(0.7885 * np.cos(k), 0.7885 * np.sin(k)), (-1.78, 1.78, -1.0, 1.0),
                    480, 270, 100, "fp32") for k in range(6)]
    ph, pd = palette(64, seed=13)
    sched = jr.Schedule(64, 16, 8, 1, 32, 0, 16, "cost")
    _, counts = jr.render_batch(frames, sched)
    _, colours = jr.render_batch(frames, sched, palette=pd)
    for c, v in zip(counts, colours):
        idx = torch.clamp(c.long(), max=63)
        assert torch.equal(pd[idx], v)


def test_plan_palette_launch_capture_and_reset():
    frames = [Frame(C1, UNIT, 200, 120, 100, "fp32"),
              Frame(complex(-0.4, 0.6), UNIT, 96, 96, 100, "fp64")]
    ph, pd = palette(101, seed=17)
    plan = jr.Plan(frames, jr.Schedule(64, 16, 8, 1, 32, 0, 16, "cost"))
    plan.launch()
    counts = [as_u32(v).view(np.int32).copy() for v in plan.views]
    plan.capture()
    plan.set_palette(pd)
    with pytest.raises(jr.JuliaError):
        plan.replay()  # the graph captured with counts was dropped
    plan.launch()
    for f, v in zip(frames, plan.views):
        np.testing.assert_array_equal(as_u32(v), expected(f, ph))
    plan.arena.fill_(-1)
    plan.capture()
    for _ in range(3):
        plan.replay()
        torch.cuda.synchronize()
        for f, v in zip(frames, plan.views):
            np.testing.assert_array_equal(as_u32(v), expected(f, ph))
        plan.arena.fill_(-1)
        torch.cuda.synchronize()
    plan.set_palette(None)
    plan.launch()
    for c, v in zip(counts, plan.views):
        np.testing.assert_array_equal(as_u32(v).view(np.int32), c)
    plan.close()


def test_palette_validation_on_device():
    _, pd = palette(16)
    with pytest.raises(ValueError):
        jr.render(C1, UNIT, 8, 8, 10, "fp64", palette=pd.view(torch.float32))
    with pytest.raises(ValueError):
        jr.render(C1, UNIT, 8, 8, 10, "fp64", palette=torch.zeros(8193, dtype=torch.int32,
                                                                   device="cuda"))


@pytest.mark.parametrize("plen", [256, 257])
def test_fp32_batch_colours_both_workgroup_shapes(plen):
    """An FP32-only batch on dispatched rows tiles: a palette of up to 256
    entries runs in one-wave workgroups (each stages its own copy), a larger
    one in four-wave workgroups.  Both against the oracle."""
    frames = [Frame(C1, UNIT, 130, 67, 100, "fp32"),
              Frame(complex(0.285, 0.01), (-1.2, 1.2, -0.9, 0.9), 97, 45, 300, "fp32"),
              Frame(0j, (-2.0, 0.6, -1.1, 1.1), 64, 50, 150, "fp32", "mandelbrot")]
    ph, pd = palette(plen, seed=19)
    sched = jr.Schedule(64, 32, 8, 0, 16, 0, 16, "cost", "rows", 48, 96)
    _, views = jr.render_batch(frames, sched, palette=pd)
    for f, v in zip(frames, views):
        np.testing.assert_array_equal(as_u32(v), expected(f, ph))
