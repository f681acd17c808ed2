"""The Mandelbrot zoom workload (Section 3: the Mandelbrot image as the
explorer's map, and deep zooms on it) in the launch the benchmark times: 64
frames of 1920 x 1080, the window from 3 down to 1e-5 wide around a boundary
point, cap 1000, FP64, one launch with the autotune cache's schedule (or the
library default).  FP64 is exact: every frame on sampled pixels, and the
widest frame whole, against the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402


def test_mandelbrot_zoom_in_the_bench_launch():
    from paper_1611_03079_amd import autotune as at
    frames = wl.mandelbrot_zoom(64)
    e = at.load_cache().get("_workloads", {}).get("mandelbrot_zoom_fp64")
    sched = jr.Schedule(**e["schedule"]) if e else None
    plan = jr.Plan(frames, sched)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(29)
    for k, (f, v) in enumerate(zip(frames, plan.views)):
        img = v.cpu().numpy()
        ii = rng.integers(0, f.width, 1500).astype(np.int32)
        jj = rng.integers(0, f.height, 1500).astype(np.int32)
        want = oracle.render_pixels(0j, f.window, f.width, f.height, f.max_iter, ii, jj, "fp64",
                                    "mandelbrot")
        np.testing.assert_array_equal(img[jj, ii], want, err_msg="frame %d" % k)
    f = frames[0]
    np.testing.assert_array_equal(plan.views[0].cpu().numpy(),
                                  oracle.render(0j, f.window, f.width, f.height, f.max_iter,
                                                "fp64", "mandelbrot"))
    plan.close()

