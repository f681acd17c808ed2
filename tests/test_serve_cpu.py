"""The serving loop's scheduling on the CPU, with a fake backend.

The fake backend renders with the oracle and completes a launch only after
a few polls, so admission, row chunking, completion order, latency accounting
and cancellation are exercised without a GPU."""
import numpy as np
import pytest

import oracle
from workloads import Frame
from paper_1611_03079_amd.serve import (ArenaAllocator, DeadlineExceeded, Overloaded,
                                        PrecisionPolicy, Server)


class FakeBackend:
    def __init__(self, capacity, polls=2, fail_launch=None):
        self.arena = np.full(capacity, -1, dtype=np.int32)
        self.polls = polls
        self.clock = 0.0
        self.launches = []
        self.fail_launch = fail_launch   # index of a launch that raises
        self.calls = 0

    def now(self):
        self.clock += 1.0
        return self.clock

    def launch(self, frames, offsets, rows, stream_idx, schedule=None):
        self.calls += 1
        if self.fail_launch == self.calls - 1:
            raise RuntimeError("launch failed")
        self.launches.append([(id(f), r) for f, r in zip(frames, rows)])
        for f, o, (r0, r1) in zip(frames, offsets, rows):
            img = oracle.render(f.c, f.window, f.width, f.height, f.max_iter, f.dtype, f.mode)
            view = self.arena[o: o + f.width * f.height].reshape(f.height, f.width)
            assert (view[r0:r1] == -1).all(), "rows rendered twice"
            view[r0:r1] = img[r0:r1]
        return [self.polls]

    def done(self, h):
        h[0] -= 1
        return h[0] < 0

    def fetch(self, offset, frame, stream_idx):
        n = frame.width * frame.height
        out = self.arena[offset: offset + n].reshape(frame.height, frame.width).copy()
        self.arena[offset: offset + n] = -1   # the range may be handed out again
        return [0], out

    def discard(self, offset, n):
        """An abandoned request's range, freed without a copy."""
        self.arena[offset: offset + n] = -1


def frames(n, w=24, h=18):
    cs = [complex(-0.8, 0.156), complex(0.285, 0.01), complex(-0.4, 0.6), complex(0.3, -0.5)]
    return [Frame(cs[k % 4], (-1.5, 1.5, -1.2, 1.2), w + k, h + (k % 3), 60 + 10 * k,
                  ("fp64", "fp32", "ff")[k % 3]) for k in range(n)]


def test_allocator_first_fit_and_merge():
    a = ArenaAllocator(100)
    x = a.alloc(30); y = a.alloc(30); z = a.alloc(30)
    assert (x, y, z) == (0, 30, 60) and a.alloc(20) is None
    a.release(y, 30)
    assert a.alloc(40) is None and a.alloc(25) == 30
    a.release(x, 30); a.release(30, 25); a.release(z, 30)
    assert a.free == [(0, 100)] and a.used == 0


def test_all_requests_complete_with_oracle_counts():
    fr = frames(7)
    b = FakeBackend(10_000)
    srv = Server(b, 10_000, step_budget=3e4)
    futs = [srv.submit(f) for f in fr]
    srv.run_until_idle(timeout=30)
    for f, fu in zip(fr, futs):
        np.testing.assert_array_equal(fu.result(), oracle.render(
            f.c, f.window, f.width, f.height, f.max_iter, f.dtype))
    assert srv.stats.completed == 7 and srv.alloc.used == 0
    # several frames share a launch, and large frames span several launches
    assert any(len(l) > 1 for l in b.launches)
    assert len(b.launches) > 1


def test_admission_by_memory_is_first_come_first_served():
    fr = frames(4, 30, 20)
    cap = 30 * 20 + 40 * 22          # room for about one frame at a time
    b = FakeBackend(cap)
    srv = Server(b, cap, step_budget=1e9)
    order = []
    futs = [srv.submit(f) for f in fr]
    for k, fu in enumerate(futs):
        fu.add_done_callback(lambda _f, k=k: order.append(k))
    srv.run_until_idle(timeout=30)
    assert order == [0, 1, 2, 3]
    assert srv.alloc.used == 0


def test_rows_are_split_over_steps_and_covered_once():
    f = Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 40, 64, 100, "fp32")
    b = FakeBackend(40 * 64)
    srv = Server(b, 40 * 64, step_budget=40 * 104 * 5)   # about 5 rows per step
    fu = srv.submit(f)
    srv.run_until_idle(timeout=30)
    rows = [r for l in b.launches for _, r in l]
    assert len(rows) >= 10
    covered = sorted(rows)
    assert covered[0][0] == 0 and covered[-1][1] == 64
    assert all(a[1] == b_[0] for a, b_ in zip(covered, covered[1:]))
    np.testing.assert_array_equal(fu.result(), oracle.render(f.c, f.window, 40, 64, 100, "fp32"))


def test_latency_is_completion_minus_arrival():
    b = FakeBackend(5000)
    srv = Server(b, 5000)
    futs = [srv.submit(f, arrival=0.5) for f in frames(3)]
    srv.run_until_idle(timeout=30)
    assert len(srv.stats.latencies) == 3
    assert all(l > 0 for l in srv.stats.latencies)
    assert srv.stats.percentile(50) <= srv.stats.percentile(99)


def test_cancelled_request_is_not_rendered():
    fr = frames(3)
    b = FakeBackend(600)           # one frame at a time fits: the others queue
    srv = Server(b, 600)
    futs = [srv.submit(f) for f in fr]
    assert futs[2].cancel()
    srv.run_until_idle(timeout=30)
    rendered = {fid for l in b.launches for fid, _ in l}
    assert id(fr[2]) not in rendered
    assert futs[0].result() is not None and futs[1].result() is not None


def rendered_rows(b, frame):
    return sorted(r for l in b.launches for fid, r in l if fid == id(frame))


def test_deadline_passes_while_queued():
    """A request whose deadline passes before it is admitted fails with
    DeadlineExceeded and is never rendered; the others complete."""
    fr = frames(3)
    b = FakeBackend(600)              # one frame at a time: the others queue
    srv = Server(b, 600, step_budget=1e9)
    futs = [srv.submit(f) for f in fr[:2]]
    late = srv.submit(fr[2], deadline=b.clock + 3)
    srv.run_until_idle(timeout=30)
    with pytest.raises(DeadlineExceeded):
        late.result(timeout=1)
    assert rendered_rows(b, fr[2]) == []
    for f, fu in zip(fr, futs):
        np.testing.assert_array_equal(fu.result(), oracle.render(
            f.c, f.window, f.width, f.height, f.max_iter, f.dtype))
    assert srv.stats.expired == 1 and srv.stats.completed == 2 and srv.alloc.used == 0


def big_frame():
    return Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 40, 64, 100, "fp32")


def test_deadline_passes_mid_frame():
    """A frame split over many steps whose deadline passes part way: it fails,
    its remaining rows are not launched, its range is freed only after its
    last launched step has finished (no row is rendered twice when the range
    is reused), and a frame submitted after it completes correctly."""
    f, g = big_frame(), frames(1)[0]
    b = FakeBackend(40 * 64 + 1000, polls=1)
    srv = Server(b, 40 * 64 + 1000, step_budget=40 * 104 * 5)   # about 5 rows per step
    fu = srv.submit(f, deadline=b.clock + 8)
    for _ in range(3):
        srv.step()
    fg = srv.submit(g)
    srv.run_until_idle(timeout=30)
    with pytest.raises(DeadlineExceeded):
        fu.result(timeout=1)
    rows = rendered_rows(b, f)
    assert 0 < len(rows) and rows[-1][1] < 64
    np.testing.assert_array_equal(fg.result(), oracle.render(g.c, g.window, g.width, g.height,
                                                             g.max_iter, g.dtype))
    assert srv.stats.expired == 1 and srv.alloc.used == 0 and (b.arena == -1).all()


def test_timeout_s_sets_every_deadline():
    b = FakeBackend(600)
    srv = Server(b, 600, step_budget=1e9, timeout_s=2.0)
    futs = [srv.submit(f) for f in frames(3)]
    srv.run_until_idle(timeout=30)
    assert isinstance(futs[2].exception(timeout=1), DeadlineExceeded)
    assert srv.stats.expired >= 1 and srv.alloc.used == 0


def test_cancel_an_admitted_request():
    """Cancelling a Future whose frame is part rendered stops its rows and
    frees its range; nothing else is disturbed."""
    f, g = big_frame(), frames(1)[0]
    b = FakeBackend(40 * 64 + 1000, polls=1)
    srv = Server(b, 40 * 64 + 1000, step_budget=40 * 104 * 5)
    fu = srv.submit(f)
    fg = srv.submit(g)
    for _ in range(3):
        srv.step()
    assert fu.cancel()
    srv.run_until_idle(timeout=30)
    assert rendered_rows(b, f)[-1][1] < 64
    np.testing.assert_array_equal(fg.result(), oracle.render(g.c, g.window, g.width, g.height,
                                                             g.max_iter, g.dtype))
    assert srv.stats.cancelled == 1 and srv.alloc.used == 0 and (b.arena == -1).all()


def test_failed_launch_fails_only_its_requests():
    """The second launch raises: the requests with rows in it fail with that
    error, the loop goes on, and later requests complete."""
    fr = frames(4, 30, 20)
    b = FakeBackend(4000, polls=1, fail_launch=1)
    srv = Server(b, 4000, step_budget=30 * 90 * 8)     # a few frames' rows per step
    futs = [srv.submit(f) for f in fr]
    srv.run_until_idle(timeout=30)
    failed = [k for k, fu in enumerate(futs) if fu.exception(timeout=1) is not None]
    assert failed and all(str(futs[k].exception()) == "launch failed" for k in failed)
    for k, (f, fu) in enumerate(zip(fr, futs)):
        if k not in failed:
            np.testing.assert_array_equal(fu.result(), oracle.render(
                f.c, f.window, f.width, f.height, f.max_iter, f.dtype))
    assert srv.stats.failed == len(failed) and srv.stats.completed == 4 - len(failed)
    assert srv.alloc.used == 0 and (b.arena == -1).all()


def test_full_queue_refuses():
    b = FakeBackend(600)
    srv = Server(b, 600, max_queue=2)
    futs = [srv.submit(f) for f in frames(3)]
    with pytest.raises(Overloaded):
        futs[2].result(timeout=1)
    srv.run_until_idle(timeout=30)
    assert futs[0].result() is not None and futs[1].result() is not None
    assert srv.stats.refused == 1


def test_oversized_frame_is_rejected():
    srv = Server(FakeBackend(100), 100)
    fu = srv.submit(Frame(0j, (-1, 1, -1, 1), 20, 20, 10, "fp32"))
    with pytest.raises(ValueError):
        fu.result(timeout=1)


def test_precision_policy():
    """The calibrated default: FP32 for windows >= 0.1 wide with caps up to
    1000, FP64 elsewhere; the specified three-way policy puts float-float
    between 1e-5 and that region."""
    p = PrecisionPolicy()
    assert p.pick(3.0, 100) == "fp32"
    assert p.pick(0.1, 1000) == "fp32"
    assert p.pick(3.0, 1001) == "fp64"
    assert p.pick(0.05, 100) == "fp64"
    assert p.pick(1e-7, 100) == "fp64"
    q = PrecisionPolicy.specified()
    assert q.pick(3.0, 100) == "fp32"
    assert q.pick(3.0, 5000) == "ff"
    assert q.pick(1e-3, 100) == "ff"
    assert q.pick(1e-5, 100) == "ff"
    assert q.pick(9e-6, 100) == "fp64"
    f = Frame(0j, (-1e-8, 1e-8, -1e-8, 1e-8), 8, 8, 100, "auto")
    srv = Server(FakeBackend(100), 100)
    srv.submit(f)
    assert f.dtype == "fp64"


def test_precision_policy_matches_the_table():
    """Every cell of the oracle's precision table that a policy routes to FP32
    or float-float has that arithmetic within 0.5% of FP64 on its probed
    pixels, for windows centred on the Julia set and for the serving
    stream's windows."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "precision_table.txt")
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert len(rows) == 36
    for pol in (PrecisionPolicy(), PrecisionPolicy.specified()):
        for kind, width, cap, px, d32, dff, _, _ in rows:
            dt = pol.pick(float(width), int(cap))
            frac = {"fp32": int(d32), "ff": int(dff), "fp64": 0}[dt] / int(px)
            assert frac <= 0.005, (kind, width, cap, dt, frac)


class TimedBackend(FakeBackend):
    """Fake backend whose launches render nothing and report a device time
    proportional to the worst-case cost of their rows (an all-interior
    workload)."""

    def __init__(self, capacity, rate):
        super().__init__(capacity, polls=0)
        self.rate = rate
        self.rows = []

    def launch(self, frames, offsets, rows, stream_idx, schedule=None):
        u = sum((r1 - r0) * Server._row_cost(f) for f, (r0, r1) in zip(frames, rows))
        self.rows.extend(rows)
        return [self.polls, u / self.rate + 15e-6]

    def seconds(self, h):
        return h[1]


def test_step_budget_follows_measured_step_times():
    """With the budget fed back from device times, steps settle at the target
    time: the learnt rate drops to the device's (here 5e10 units/s) after the
    first full step, and a large frame is then split into steps of about the
    target length."""
    from paper_1611_03079_amd.serve import StepRate
    f = Frame(complex(-0.8, 0.156), (-1.5, 1.5, -1.5, 1.5), 200, 4000, 3000, "fp64")
    b = TimedBackend(200 * 4000, rate=5e10)
    srv = Server(b, 200 * 4000, step_target_s=1e-3, rate=StepRate(prior=4e11), keep_log=True)
    srv.submit(f)
    srv.run_until_idle(timeout=60)
    assert abs(srv.rate.rate - 5e10) / 5e10 < 1e-6
    times = [r.seconds for r in srv.log]
    # the first steps use the prior (too large); once learnt, every full
    # step lasts about the target
    assert times[0] > 2e-3
    full = [t for r, t in zip(srv.log[2:], times[2:]) if r.units >= 0.5 * srv.step_budget]
    assert len(full) >= 10 and all(abs(t - 1e-3) < 0.1e-3 for t in full)
    # the rows are covered once and the row costs have no cap
    rows = sorted(b.rows)
    assert rows[0][0] == 0 and rows[-1][1] == 4000
    assert all(a[1] == c[0] for a, c in zip(rows, rows[1:]))
    assert Server._row_cost(f) == 200 * 3004 * 2.1


def test_step_rate_rises_slowly_and_is_capped():
    from paper_1611_03079_amd.serve import StepRate
    r = StepRate(prior=1e12, ceiling=3e12, growth=1.1)
    r.update(1e12 * 1e-3, 1e-3 + 15e-6)        # as fast as the prior
    assert abs(r.rate - 1e12) < 1e3
    for _ in range(5):
        r.update(1e20, 1e-3)                   # light steps: at most 10% up each
    assert abs(r.rate - 1e12 * 1.1 ** 5) < 1e6
    for _ in range(50):
        r.update(1e20, 1e-3)
    assert r.rate == 3e12
    r.update(2e11 * 1e-3, 1e-3 + 15e-6)        # a heavy step: down at once
    assert abs(r.rate - 2e11) < 1e3
