"""GPU parity of the two-parameter rational maps Z^d + C + lambda / Z^d
against the oracle.

Launches holding such frames run the rows kernel (schedules asking for the
tiled or hybrid stream are carried over to it) or the batched plain kernel;
every frame must equal the oracle's image bit for bit in FP64 and FP32, with
escape absorbing (blocked tests) and not (a test on every iteration), mixed
with polynomial frames in one launch, and with the fused colour store.
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
    jr.Schedule(64, 16, 8, 0, 16, 0, 16, "cost", "rows", 8),
    jr.Schedule(64, 64, 8, 0, 16, 0, 16, "cost", "rows", 48, 32),
    jr.Schedule(37, 5, 4, 0, 32, 1, 8, "table", "rows", 2),
    jr.Schedule(kernel="plain", order="table"),
    jr.Schedule(16, 16, 8, 1, 32, 0, 16, "cost"),                # carried over to rows
    jr.Schedule(64, 16, 8, 0, 16, 1, 16, "cost", "hybrid", 300),  # carried over to rows
]


def ref(f: Frame):
    if f.lam is None:
        return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode,
                             f.degree)
    return oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, "julia",
                         f.degree, lam=f.lam)


def R(c, lam, win, W, H, cap, dtype, d=2):
    return Frame(c, win, W, H, cap, dtype, "julia", d, lam)


def frames_mixed():
    return [
        R(complex(-0.55, 0.1), complex(-0.02, 0.01), (-1.5, 1.5, -1.2, 1.2), 97, 61, 150, "fp64"),
        R(complex(-0.1, 0.65), complex(0.005, 0.005), (-1.3, 1.1, -0.9, 1.0), 80, 66, 200,
          "fp32", 3),
        Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 64, 48, 100, "fp32"),
        R(complex(0.2, 0.3), complex(0.01, -0.01), (-1.4, 1.4, -1.4, 1.4), 45, 33, 120, "fp64", 4),
        # escape not absorbing (|C| + |lambda| / 4 > 1.9): a test on every iteration
        R(complex(1.7, 0.2), complex(0.9, -0.3), (-1.6, 1.6, -1.6, 1.6), 40, 40, 60, "fp32"),
        R(complex(-0.75, 0.1), complex(0.002, 0.001), (-1.3, 1.3, -1.1, 1.1), 33, 129, 80,
          "fp64", 4),
        Frame(complex(0.4, 0.3), (-1.3, 1.3, -1.2, 1.2), 50, 40, 90, "fp32", "julia", 3),
    ]


@pytest.mark.parametrize("degree", [2, 3, 4, 7])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_single_image(dtype, degree):
    c, lam = complex(-0.55, 0.1), complex(-0.02, 0.01)
    win = (-1.5, 1.5, -1.2, 1.2)
    want = oracle.render(c, win, 131, 67, 120, dtype, "julia", degree, lam=lam)
    assert len(np.unique(want)) >= 5
    for plain in (False, True):
        got = jr.render(c, win, 131, 67, 120, dtype, degree=degree, lam=lam, plain=plain)
        torch.cuda.synchronize()
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


def test_pole_and_exact_orbits_on_the_device():
    """Dyadic grids whose orbits are exact: the one-column grid over
    Re[-1, 1] x Im[-2, 2] has the pixels +-i, which with C = 0 and
    lambda = -1 step to the pole 0 and then to 0/0 (not a number: escaped,
    count 2, as the oracle's hand-worked orbit); fixed points where
    lambda / W cancels C; and 4 x 4 grids over [-2, 2]^2 (centres +-0.5,
    +-1.5)."""
    cases = [(0j, complex(-1.0, 0.0), (-1.0, 1.0, -2.0, 2.0), 1, 2, [[2], [2]]),
             (complex(-1.0, -1.0), complex(1.0, 1.0), (-2.0, 2.0, -2.0, 2.0), 4, 4, None),
             (0j, complex(-0.25, 0.0), (-2.0, 2.0, -2.0, 2.0), 4, 4, None),
             (complex(-1.0, 0.0), complex(1.0, 0.0), (-2.0, 2.0, -2.0, 2.0), 4, 4, None)]
    for c, lam, win, W, H, hand in cases:
        for dtype in ("fp64", "fp32"):
            want = oracle.render(c, win, W, H, 100, dtype, "julia", 2, lam=lam)
            if hand is not None:
                assert want.tolist() == hand
            got = jr.render(c, win, W, H, 100, dtype, lam=lam)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy(), want, err_msg=str((c, lam)))


def test_colours_of_rational_maps():
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


def test_large_rational_frame_sampled():
    f = R(complex(-0.1, 0.65), complex(0.005, 0.005), (-1.3, 1.3, -1.3, 1.3), 2048, 2048, 400,
          "fp64", 2)
    out = jr.render(f.c, f.window, f.width, f.height, f.max_iter, "fp64", lam=f.lam)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    ii = rng.integers(0, f.width, 4000).astype(np.int32)
    jj = rng.integers(0, f.height, 4000).astype(np.int32)
    want = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, "fp64",
                                "julia", 2, lam=f.lam)
    np.testing.assert_array_equal(out.cpu().numpy()[jj, ii], want)


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
def test_rational_path_in_the_bench_launch(dtype):
    """The benchmark's rational workload: 32 frames of 1920 x 1080 of
    Z^2 + C_k + lam_k / Z^2 in one launch with the autotune cache's schedule
    (or the library default), each frame on 2000 sampled pixels against the
    oracle, and every 8th frame whole."""
    import workloads as wl
    from paper_1611_03079_amd import autotune as at
    frames = wl.rational_path(32, 2, dtype=dtype)
    e = at.load_cache().get("_workloads", {}).get("rational_deg2_" + dtype)
    sched = jr.Schedule(**e["schedule"]) if e else None
    plan = jr.Plan(frames, sched)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    for k, (f, v) in enumerate(zip(frames, plan.views)):
        img = v.cpu().numpy()
        if k % 8 == 0:
            np.testing.assert_array_equal(img, ref(f), err_msg="frame %d" % k)
            continue
        ii = rng.integers(0, f.width, 2000).astype(np.int32)
        jj = rng.integers(0, f.height, 2000).astype(np.int32)
        want = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, dtype,
                                    "julia", 2, lam=f.lam)
        np.testing.assert_array_equal(img[jj, ii], want, err_msg="frame %d" % k)
    plan.close()
