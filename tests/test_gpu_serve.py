"""Serving loop on the GPU: every result equals the same request alone.

Requests of different sizes, caps and (policy-picked) dtypes are admitted while
others run, share launches and overlap on two streams; scheduling never changes
a count, so each result must equal julia_render of the request by itself, and
the oracle on sampled pixels."""
import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import Frame

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_1611_03079_amd as jr  # noqa: E402
from paper_1611_03079_amd.serve import GpuBackend, PrecisionPolicy, Server, run_open_loop  # noqa: E402,E501

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


def test_deadlines_and_cancellation_on_the_device():
    """A large slow request whose deadline passes while its rows are in
    flight fails with DeadlineExceeded and stops being rendered; a cancelled
    one likewise; the requests around them, which reuse the freed arena, equal
    the same requests alone."""
    from paper_1611_03079_amd.serve import DeadlineExceeded
    import time
    slow = Frame(complex(-0.8, 0.156), (-0.61, -0.59, 0.09, 0.11), 640, 480, 20000, "fp64")
    slow2 = Frame(complex(-0.8, 0.156), (-0.60, -0.58, 0.10, 0.12), 640, 480, 20000, "fp64")
    small = [r.frame for r in _stream(12, 21)]
    cap = 2 * 640 * 480 + 2 * 320 * 240
    b = GpuBackend(cap)
    srv = Server(b, cap, step_budget=2e6)
    f_slow = srv.submit(slow, deadline=time.perf_counter() + 0.002)
    f_cancel = srv.submit(slow2)
    futs = [srv.submit(f) for f in small[:6]]
    for _ in range(4):
        srv.step()
    assert f_cancel.cancel()
    futs += [srv.submit(f) for f in small[6:]]
    srv.run_until_idle(timeout=100)
    with pytest.raises(DeadlineExceeded):
        f_slow.result(timeout=1)
    assert f_cancel.cancelled()
    assert srv.stats.expired == 1 and srv.stats.cancelled == 1
    assert srv.stats.completed == len(small) and srv.alloc.used == 0
    for f, fu in zip(small, futs):
        np.testing.assert_array_equal(fu.result().cpu().numpy(), _alone(f))


def test_open_loop_arrivals():
    reqs = _stream(40, 9)
    cap = 4 * 320 * 240
    srv = Server(GpuBackend(cap), cap, step_budget=4e6, copy_out=False)
    stats = run_open_loop(srv, reqs, drain_timeout=100)
    assert stats.completed == len(reqs)
    assert stats.percentile(50) <= stats.percentile(99)
    assert stats.percentile(99) < 100.0


def test_admission_during_a_step_and_overlapping_steps():
    """Continuous batching on the device: a request that arrives while a
    heavy step runs is admitted at once, launched in the next step on the
    other stream while the first is still running (host view), and the two
    steps overlap on the device (the second step's start event precedes the
    first step's end event).  Both results equal the requests alone."""
    heavy = Frame(complex(-0.1, 0.1), (-1.2, 1.2, -0.9, 0.9), 1920, 1080, 4000, "fp64")
    light = Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 320, 240, 200, "fp32")
    cap = heavy.pixels + light.pixels
    b = GpuBackend(cap)
    srv = Server(b, cap, step_budget=1e15, keep_log=True)
    fh = srv.submit(heavy)
    srv.step()                                  # step 0: the whole heavy frame
    assert len(srv.log) == 1 and not b.done(srv.log[0].handle)
    fl = srv.submit(light)                      # arrives while step 0 runs
    srv.step()                                  # admitted, launched as step 1
    assert len(srv.log) == 2
    s0, s1 = srv.log
    rid_light = s1.rids[0]
    t_admit, inflight = srv.admitted_at[rid_light]
    assert inflight == [0] and s1.inflight_at_launch == [0]
    assert s0.stream != s1.stream
    srv.run_until_idle(timeout=60)
    # device timeline: step 1 started before step 0 ended
    assert b.between(s1.handle, s0.handle) > 0
    np.testing.assert_array_equal(fh.result().cpu().numpy(), _alone(heavy))
    np.testing.assert_array_equal(fl.result().cpu().numpy(), _alone(light))


def test_step_budget_is_learnt_on_the_device():
    """With no fixed budget, the loop learns from step times how much
    worst-case work fits its target step time: heavy all-interior frames are
    split over several steps, each lasting about the target or less."""
    frames = [Frame(complex(-0.1, 0.1), (-0.5, 0.5, -0.5, 0.5), 640, 480, 3000, "fp64")
              for _ in range(16)]
    cap = sum(f.pixels for f in frames)
    srv = Server(GpuBackend(cap), cap, step_target_s=1e-3, keep_log=True)
    futs = [srv.submit(f) for f in frames]
    srv.run_until_idle(timeout=60)
    assert srv.stats.completed == 16 and srv.rate.samples >= 3
    times = sorted(r.seconds for r in srv.log[4:])
    # after the first steps, the median step is near the target, never far
    # beyond it (two steps may share the device, so allow 3x at the top)
    assert times and times[len(times) // 2] < 2.0e-3 and times[-1] < 3.0e-3
    want = _alone(frames[0])
    for fu in futs:
        np.testing.assert_array_equal(fu.result().cpu().numpy(), want)


def _routed_cells(kind, policy):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "precision_table.txt")
    out = []
    for k, width, cap, *_ in (l.split() for l in open(path) if not l.startswith("#")):
        dt = policy.pick(float(width), int(cap))
        if k == kind and dt != "fp64":
            out.append((float(width), int(cap), dt))
    return out


def _check_cells(kind, cells, windows):
    """For each (width, cap, dtype) cell: the first `windows` windows of the
    cell rendered whole on the GPU in FP64 and in dtype; on their probed
    pixels both equal the oracle, and over the whole windows the fraction of
    pixels whose dtype count differs from FP64 is within the stated 0.5%."""
    from concurrent.futures import ThreadPoolExecutor
    report = []
    pool = ThreadPoolExecutor(16)
    for width, cap, dt in cells:
        wins = wl.probe_windows(kind, width, cap)[:windows]
        print("precision cell %s width %g cap %d %s" % (kind, width, cap, dt), flush=True)
        imgs = {}
        for d in ("fp64", dt):
            _, views = jr.render_batch([Frame(w.frame.c, w.frame.window, w.frame.width,
                                              w.frame.height, cap, d) for w in wins])
            imgs[d] = [v.cpu().numpy() for v in views]

        def probe(args):
            w, d = args
            f = w.frame
            return oracle.render_pixels(f.c, f.window, f.width, f.height, cap,
                                        np.asarray(w.ii, np.int32), np.asarray(w.jj, np.int32), d)
        for d in ("fp64", dt):
            want = list(pool.map(probe, [(w, d) for w in wins]))
            for img, w, ref_ in zip(imgs[d], wins, want):
                np.testing.assert_array_equal(img[w.jj, w.ii], ref_, err_msg="%s %g %d %s" % (
                    kind, width, cap, d))
        diff = sum(int((a != b).sum()) for a, b in zip(imgs[dt], imgs["fp64"]))
        frac = diff / sum(w.frame.pixels for w in wins)
        report.append("%s %g %d %s %.4f%%" % (kind, width, cap, dt, 100 * frac))
        assert frac <= 0.005, report[-1]
    pool.shutdown()
    print("; ".join(report), flush=True)


@pytest.mark.parametrize("kind", ["serving", "boundary"])
def test_precision_bound_of_the_calibrated_policy(kind):
    """Every cell the default policy sends to FP32 (windows >= 0.1 wide, caps
    up to 1000): 8 whole 640x480 windows per cell, FP32 within 0.5% of FP64."""
    cells = _routed_cells(kind, PrecisionPolicy())
    assert cells and {dt for *_, dt in cells} == {"fp32"}
    _check_cells(kind, cells, 8)


@pytest.mark.parametrize("kind", ["serving", "boundary"])
def test_precision_bound_of_the_float_float_cells(kind):
    """Every cell the three-way policy sends to float-float (1e-5 <= width,
    outside the FP32 region): whole windows, 4 per cell with caps up to 1000
    and 2 with cap 5000 (float-float runs at about a tenth of FP64's rate),
    float-float within 0.5% of FP64."""
    cells = [c for c in _routed_cells(kind, PrecisionPolicy.specified()) if c[2] == "ff"]
    assert cells
    _check_cells(kind, [c for c in cells if c[1] <= 1000], 4)
    _check_cells(kind, [c for c in cells if c[1] > 1000], 2)
