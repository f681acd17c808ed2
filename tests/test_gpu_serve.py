"""Serving loop on the GPU: every result equals the same request alone.

Requests of different sizes, caps and (policy-picked) dtypes are admitted while
others run, share launches and overlap on two streams; scheduling never changes
a count, so each result must equal julia_render of the request by itself, and
the oracle on sampled pixels."""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402
from paper_1611_03079_amd.serve import GpuBackend, Server, run_open_loop  # noqa: E402

SIZES = ((160, 120), (320, 240), (256, 144))


def _stream(n, seed):
    return wl.serving_stream(seed, 2000.0, n, sizes=SIZES, cap_hi=800, width_lo=1e-8)


def _alone(f):
    out = jr.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_results_alone_equal_in_mix():
    reqs = _stream(30, 5)
    cap = 3 * 320 * 240
    srv = Server(GpuBackend(cap), cap, step_budget=4e6)
    futs = [srv.submit(r.frame) for r in reqs]
    srv.run_until_idle(timeout=100)
    assert srv.stats.completed == len(reqs) and srv.alloc.used == 0
    assert srv.stats.steps > 3
    dts = set()
    rng = np.random.default_rng(0)
    for r, fu in zip(reqs, futs):
        f = r.frame
        dts.add(f.dtype)
        got = fu.result().cpu().numpy()
        np.testing.assert_array_equal(got, _alone(f))
        ii = rng.integers(0, f.width, 200).astype(np.int32)
        jj = rng.integers(0, f.height, 200).astype(np.int32)
        want = oracle.render_pixels(f.c, f.window, f.width, f.height, f.max_iter, ii, jj, f.dtype)
        np.testing.assert_array_equal(got[jj, ii], want)
    assert len(dts) >= 2


def test_open_loop_arrivals():
    reqs = _stream(40, 9)
    cap = 4 * 320 * 240
    srv = Server(GpuBackend(cap), cap, step_budget=4e6, copy_out=False)
    stats = run_open_loop(srv, reqs, drain_timeout=100)
    assert stats.completed == len(reqs)
    assert stats.percentile(50) <= stats.percentile(99)
    assert stats.percentile(99) < 100.0
