"""Continuous-batching request loop for interactive exploration.

The paper's application renders a Julia image for the parameter the user is
moving (Sections 2 and 3: real-time full-screen frames, parameter paths, deep
zooms).  This loop serves a stream of such requests on one GPU:

  * requests arrive at any time (submit() returns a Future);
  * a request is admitted when its counts fit in the device output arena
    (memory-based admission, first come first served);
  * every step takes rows from all admitted requests, oldest first, up to a
    work budget, and renders them in ONE launch of the batch kernel (frames of
    different sizes, caps and dtypes together; a large frame is split over
    several steps by row ranges).  The budget is fed back from measured step
    times: a row costs its worst case (every pixel runs to the cap), and the
    rate at which the device clears such work is learnt from the device time
    of finished steps, so a step lasts about `step_target_s` at most and a new
    arrival starts within one step;
  * two steps are kept in flight on two streams, so work admitted while
    others run overlaps with them on the device;
  * a request completes when the step holding its last rows has finished; its
    counts are copied out of the arena and the arena range is freed;
  * latency = completion time - arrival time; p50/p99 and throughput are kept;
  * failures stay with their requests: a request may carry a deadline (it
    fails with DeadlineExceeded once the deadline passes before its last rows
    are rendered, and its remaining rows are not rendered), a cancelled
    Future's rows stop being scheduled, a full queue refuses new requests
    with Overloaded, and a launch that raises fails only the requests of that
    step.  An abandoned request's arena range is freed once no step in
    flight still writes into it.

The arithmetic of each frame is picked by a precision policy from its window
width and cap.  Scheduling never changes a count, so every result equals the
same request rendered alone.
"""
import collections
import math
import threading
import time
from concurrent.futures import Future, InvalidStateError
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional

# Relative cost of one pixel-iteration by arithmetic, in FP32 units, for the
# step budget: what the batched kernels take per pixel-iteration on the
# parameter path (FP64 about 2.1x FP32, float-float about 7.3x), rounded up
# for float-float, whose long orbits dominate a step that holds them.  The
# budget's scale is learnt from measured step times; only these ratios are
# fixed.
DTYPE_COST = {"fp32": 1.0, "fp64": 2.1, "ff": 10.0}


class DeadlineExceeded(TimeoutError):
    """The request's deadline passed before its image was rendered."""


def _fail(fut: Future, exc: BaseException):
    """Fail a Future unless it is already done or the client cancelled it
    (which may happen at any moment from another thread)."""
    try:
        if not fut.done():
            fut.set_exception(exc)
    except InvalidStateError:
        pass


class Overloaded(RuntimeError):
    """The server's queue was full when the request arrived."""


@dataclass
class PrecisionPolicy:
    """dtype by window width and cap: FP32 where its counts stay within the
    stated bound of FP64's, float-float for narrower windows down to
    `ff_min_width`, FP64 below.

    The thresholds come from the measured precision table (FP32 and
    float-float against FP64, windows centred on the Julia set, the hardest
    case): FP32 differs from FP64 on at most 0.32% of pixels for windows at
    least 0.1 wide with caps up to 1000, and on more (0.69% to 93%) for
    narrower windows or larger caps; float-float on at most 0.28% down to
    1e-9.  The default routes everything that FP32 does not cover to FP64:
    on MI355X FP64 is exact and costs about 2.1 times FP32 per iteration on
    the parameter path, float-float about 7.3 times.  `specified()` is the three-way policy with float-float between
    1e-5 and the FP32 region."""
    fp32_min_width: float = 0.1
    fp32_max_iter: int = 1000
    ff_min_width: float = math.inf

    @staticmethod
    def specified() -> "PrecisionPolicy":
        return PrecisionPolicy(ff_min_width=1e-5)

    def pick(self, width: float, max_iter: int) -> str:
        if width >= self.fp32_min_width and max_iter <= self.fp32_max_iter:
            return "fp32"
        if width >= self.ff_min_width:
            return "ff"
        return "fp64"


class StepRate:
    """The rate (worst-case cost units per second) at which the device clears
    a step, learnt from finished steps.  A row's cost assumes every pixel runs
    to the cap, so a step's measured rate is at least the device's true rate
    and equals it when the rows are all interior.  The estimate follows the
    lower envelope of the measured rates: it drops to any lower measurement at
    once and rises by at most `growth` per step, and it never exceeds `ceiling`
    (the FP32 issue-rate limit of MI355X in these units), so a heavy step
    after a run of light ones overruns its target by a bounded factor."""

    def __init__(self, prior: float = 2.0e12, ceiling: float = 9.0e12, growth: float = 1.05,
                 fixed_s: float = 15e-6):
        self.rate = prior
        self.ceiling = ceiling
        self.growth = growth
        self.fixed_s = fixed_s   # launch and event overhead of one step
        self.samples = 0

    def update(self, units: float, seconds: float):
        busy = seconds - self.fixed_s
        if units <= 0 or busy <= 0:
            return
        self.samples += 1
        self.rate = min(self.ceiling, self.rate * self.growth, units / busy)


class ArenaAllocator:
    """First-fit allocator of element ranges in [0, capacity)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free = [(0, self.capacity)]  # sorted (offset, length)
        self.used = 0

    def alloc(self, n: int) -> Optional[int]:
        for k, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int):
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


@dataclass
class _Req:
    rid: int
    frame: object            # has c, window, width, height, max_iter, dtype, mode
    arrival: float
    future: Future
    offset: int = -1
    next_row: int = 0
    last_step: int = -1      # step that holds the frame's last rows
    done_rows: int = 0
    deadline: float = math.inf
    launched: int = 0        # steps in flight that hold some of its rows
    dead: bool = False       # abandoned: expired, cancelled or failed


@dataclass
class Stats:
    """Latency and throughput of a run.  `latencies` holds the completed
    requests' latencies; `unfinished` the requests still pending when the run
    was cut off, each at the time it had waited by then (a lower bound of its
    latency).  Percentiles count both, so a loop that falls behind cannot
    report only the requests it managed to finish."""
    latencies: List[float] = field(default_factory=list)
    unfinished: List[float] = field(default_factory=list)
    completed: int = 0
    expired: int = 0         # failed with DeadlineExceeded
    cancelled: int = 0       # cancelled by the client before completion
    failed: int = 0          # failed by a launch that raised
    refused: int = 0         # refused at submission (full queue)
    pixels: int = 0
    steps: int = 0
    t_first: float = math.inf
    t_last: float = 0.0

    @property
    def offered(self) -> int:
        return self.completed + len(self.unfinished)

    @property
    def saturated(self) -> bool:
        """Requests were left pending: the offered rate exceeded what the
        loop sustained, and the percentiles are lower bounds."""
        return len(self.unfinished) > 0

    def percentile(self, q: float, completed_only: bool = False) -> float:
        xs = self.latencies if completed_only else self.latencies + self.unfinished
        if not xs:
            return math.nan
        xs = sorted(xs)
        k = min(len(xs) - 1, max(0, int(math.ceil(q / 100.0 * len(xs))) - 1))
        return xs[k]


class GpuBackend:
    """libjulia.so on the current CUDA device: device arena, two streams.  A
    launch is bracketed by timing events on its stream; their times give the
    step's device time (the budget's feedback) and show steps overlapping."""

    def __init__(self, arena_elements: int, streams: int = 2):
        import torch
        import paper_1611_03079_amd as jr
        self.torch, self.jr = torch, jr
        self.arena = torch.empty(int(arena_elements), dtype=torch.int32, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(streams)]

    def now(self) -> float:
        return time.perf_counter()

    def launch(self, frames, offsets, rows, stream_idx: int, schedule=None):
        st = self.streams[stream_idx]
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        self.jr.render_batch(frames, schedule, arena=self.arena, offsets=offsets, rows=rows,
                             stream=st)
        ev1.record(st)
        return (ev0, ev1)

    def done(self, handle) -> bool:
        return handle[1].query() if isinstance(handle, tuple) else handle.query()

    def seconds(self, handle) -> float:
        """Device time of a finished launch."""
        return handle[0].elapsed_time(handle[1]) * 1e-3

    def between(self, a, b) -> float:
        """Device time from the start event of launch a to the end event of
        launch b (negative when b ended before a started)."""
        return a[0].elapsed_time(b[1]) * 1e-3

    def fetch(self, offset: int, frame, stream_idx: int):
        st = self.streams[stream_idx]
        n = frame.width * frame.height
        with self.torch.cuda.stream(st):
            out = self.arena[offset: offset + n].view(frame.height, frame.width).clone()
            ev = self.torch.cuda.Event()
            ev.record(st)
        return ev, out


@dataclass
class StepRecord:
    """One launch of the loop, kept for inspection (tests, reports)."""
    step: int
    stream: int
    rids: List[int]
    units: float              # worst-case cost of its rows
    t_launch: float           # host clock when it was enqueued
    inflight_at_launch: List[int]  # steps not yet finished at that moment
    handle: object = None
    seconds: float = math.nan  # device time, once finished


class Server:
    def __init__(self, backend, arena_elements: int, step_budget: Optional[float] = None,
                 max_inflight: int = 2, policy: Optional[PrecisionPolicy] = None,
                 copy_out: bool = True, schedule=None, step_target_s: float = 2e-3,
                 rate: Optional[StepRate] = None, keep_log: bool = False,
                 max_queue: Optional[int] = None, timeout_s: Optional[float] = None):
        self.b = backend
        # requests waiting for admission beyond this many are refused
        self.max_queue = max_queue
        # default deadline of a request: its arrival plus this many seconds
        self.timeout_s = timeout_s
        self.alloc = ArenaAllocator(arena_elements)
        # a fixed budget (cost units per step), or None: step_target_s times
        # the learnt rate
        self.fixed_budget = step_budget
        self.step_target_s = step_target_s
        self.rate = rate or StepRate()
        self.keep_log = keep_log
        self.log: List[StepRecord] = []
        self.admitted_at: Dict[int, tuple] = {}   # rid -> (host time, steps in flight)
        self.max_inflight = max_inflight
        self.policy = policy or PrecisionPolicy()
        self.copy_out = copy_out
        self.schedule = schedule
        self.queue: Deque[_Req] = collections.deque()
        self.active: List[_Req] = []
        self.inflight: Deque = collections.deque()   # (step id, handle, [reqs ending here])
        self.fetching: List = []                     # (handle, req, result)
        self.stats = Stats()
        self.lock = threading.Lock()
        self.step_id = 0
        self._rid = 0
        self._stop = False
        self._thread = None

    # ------------------------------------------------------------- client side
    def submit(self, frame, arrival: Optional[float] = None,
               deadline: Optional[float] = None) -> Future:
        """Queue a request.  ``deadline``: time on the backend's clock by
        which the image must be rendered (default: arrival + timeout_s, or
        none); past it the Future fails with DeadlineExceeded.  A frame whose
        dtype is "auto" (or None) gets the policy's pick written into its
        dtype field, so the caller can see which arithmetic rendered it."""
        fut = Future()
        if frame.width * frame.height > self.alloc.capacity:
            fut.set_exception(ValueError("frame larger than the output arena"))
            return fut
        if getattr(frame, "dtype", None) in (None, "auto"):
            w = frame.window[1] - frame.window[0]
            frame.dtype = self.policy.pick(w, frame.max_iter)
        t = self.b.now() if arrival is None else arrival
        if deadline is None:
            deadline = math.inf if self.timeout_s is None else t + self.timeout_s
        with self.lock:
            if self.max_queue is not None and len(self.queue) >= self.max_queue:
                self.stats.refused += 1
                fut.set_exception(Overloaded("%d requests already waiting" % len(self.queue)))
                return fut
            self._rid += 1
            self.queue.append(_Req(self._rid, frame, t, fut, deadline=deadline))
        return fut

    def pending(self) -> int:
        with self.lock:
            return len(self.queue) + len(self.active) + len(self.fetching)

    def censor(self, t: float):
        """Record every request still pending at time t as unfinished, with
        the latency it has accumulated by t (the run is over)."""
        with self.lock:
            waiting = list(self.queue) + [r for r in self.active if not r.dead]
        for r in waiting:
            self.stats.unfinished.append(t - r.arrival)
            self.stats.t_first = min(self.stats.t_first, r.arrival)

    # ------------------------------------------------------------- scheduler
    def _abandon(self, r: _Req, exc: Optional[BaseException]):
        """Stop rendering r: fail its Future with exc (None: it was cancelled)
        and free its arena range once no step in flight writes into it."""
        if r.dead:
            return
        r.dead = True
        if exc is None:
            self.stats.cancelled += 1
        else:
            if isinstance(exc, DeadlineExceeded):
                self.stats.expired += 1
            else:
                self.stats.failed += 1
            _fail(r.future, exc)
        self._reap(r)

    def _reap(self, r: _Req):
        if r.dead and r.launched == 0 and r.offset >= 0:
            n = r.frame.width * r.frame.height
            discard = getattr(self.b, "discard", None)
            if discard is not None:
                discard(r.offset, n)
            with self.lock:
                if r in self.active:
                    self.active.remove(r)
                self.alloc.release(r.offset, n)
            r.offset = -1

    def _expire(self):
        """Drop queued requests that were cancelled or are past their
        deadline; abandon admitted ones likewise (unless their last rows are
        already rendered and being copied out)."""
        with self.lock:
            timed = any(r.deadline < math.inf for r in self.queue) or \
                any(r.deadline < math.inf for r in self.active)
        now = self.b.now() if timed else -math.inf
        with self.lock:
            keep = collections.deque()
            for r in self.queue:
                if r.future.cancelled():
                    self.stats.cancelled += 1
                elif now > r.deadline:
                    self.stats.expired += 1
                    _fail(r.future, DeadlineExceeded(
                        "request %d: deadline passed while queued" % r.rid))
                else:
                    keep.append(r)
            self.queue = keep
            active = list(self.active)
        fetching = {id(r) for _, r, _ in self.fetching}
        for r in active:
            if r.dead or id(r) in fetching or (r.next_row >= r.frame.height and r.launched == 0):
                continue
            if r.future.cancelled():
                self._abandon(r, None)
            elif now > r.deadline:
                self._abandon(r, DeadlineExceeded(
                    "request %d: deadline passed after %d of %d rows"
                    % (r.rid, r.next_row, r.frame.height)))

    def _admit(self):
        with self.lock:
            while self.queue:
                r = self.queue[0]
                if r.future.cancelled():
                    self.stats.cancelled += 1
                    self.queue.popleft()
                    continue
                off = self.alloc.alloc(r.frame.width * r.frame.height)
                if off is None:
                    break   # first come first served: the head waits for memory
                r.offset = off
                self.active.append(self.queue.popleft())
                if self.keep_log:
                    self.admitted_at[r.rid] = (self.b.now(), [s[0] for s in self.inflight])

    @staticmethod
    def _row_cost(f) -> float:
        """Worst-case cost of one row: every pixel runs to the cap."""
        return f.width * (4.0 + f.max_iter) * DTYPE_COST[f.dtype]

    @property
    def step_budget(self) -> float:
        if self.fixed_budget is not None:
            return self.fixed_budget
        return self.step_target_s * self.rate.rate

    def _build_step(self):
        frames, offsets, rows, ending, rids = [], [], [], [], []
        units = 0.0
        budget = self.step_budget
        reqs = []
        for r in self.active:
            if r.dead or r.next_row >= r.frame.height:
                continue
            f = r.frame
            rc = self._row_cost(f)
            take = max(1, min(f.height - r.next_row, int(budget // rc)))
            frames.append(f)
            offsets.append(r.offset)
            rows.append((r.next_row, r.next_row + take))
            rids.append(r.rid)
            reqs.append(r)
            r.next_row += take
            if r.next_row >= f.height:
                r.last_step = self.step_id
                ending.append(r)
            budget -= take * rc
            units += take * rc
            if budget <= 0:
                break
        return frames, offsets, rows, ending, rids, units, reqs

    def step(self) -> bool:
        """One scheduler pass; returns True when it did anything."""
        busy = False
        self._expire()
        self._admit()
        if len(self.inflight) < self.max_inflight:
            frames, offsets, rows, ending, rids, units, reqs = self._build_step()
            if frames:
                sidx = self.step_id % self.max_inflight
                t = self.b.now()
                before = [s[0] for s in self.inflight]
                try:
                    h = self.b.launch(frames, offsets, rows, sidx, self.schedule)
                except Exception as e:   # the step's requests fail; the loop goes on
                    for r in reqs:
                        self._abandon(r, e)
                    return True
                for r in reqs:
                    r.launched += 1
                rec = StepRecord(self.step_id, sidx, rids, units, t, before, h)
                self.inflight.append((self.step_id, sidx, h, ending, rec, reqs))
                if self.keep_log:
                    self.log.append(rec)
                self.step_id += 1
                self.stats.steps += 1
                busy = True
        while self.inflight and self.b.done(self.inflight[0][2]):
            _, sidx, h, ending, rec, reqs = self.inflight.popleft()
            for r in reqs:
                r.launched -= 1
                self._reap(r)
            seconds = getattr(self.b, "seconds", None)
            if seconds is not None:
                rec.seconds = seconds(h)
                # only steps that used most of their budget say how fast the
                # device clears work; small ones are mostly launch overhead
                if self.fixed_budget is None and rec.units >= 0.5 * self.step_budget:
                    self.rate.update(rec.units, rec.seconds)
            for r in ending:
                if r.dead:
                    continue
                if self.copy_out:
                    h, out = self.b.fetch(r.offset, r.frame, sidx)
                else:
                    h, out = None, None
                self.fetching.append((h, r, out))
            busy = True
        keep = []
        for h, r, out in self.fetching:
            if h is None or self.b.done(h):
                t = self.b.now()
                self.stats.latencies.append(t - r.arrival)
                self.stats.completed += 1
                self.stats.pixels += r.frame.width * r.frame.height
                self.stats.t_first = min(self.stats.t_first, r.arrival)
                self.stats.t_last = max(self.stats.t_last, t)
                with self.lock:
                    self.active.remove(r)
                    self.alloc.release(r.offset, r.frame.width * r.frame.height)
                try:
                    if not r.future.done():
                        r.future.set_result(out)
                except InvalidStateError:
                    pass  # cancelled by the client just now
                busy = True
            else:
                keep.append((h, r, out))
        self.fetching = keep
        return busy

    def run_until_idle(self, timeout: float = 60.0):
        t_end = time.perf_counter() + timeout
        while self.pending() and time.perf_counter() < t_end:
            if not self.step():
                time.sleep(0.0001)
        if self.pending():
            raise TimeoutError("requests still pending after %.1f s" % timeout)

    def start(self):
        def loop():
            while not self._stop:
                if not self.step():
                    time.sleep(0.0001)
        self._thread = threading.Thread(target=loop, daemon=True)
        self._thread.start()

    def stop(self):
        self._stop = True
        if self._thread:
            self._thread.join()


def run_open_loop(server: Server, requests, drain_timeout: float = 60.0) -> Stats:
    """Submit requests at their scheduled arrival times (open loop: latency is
    measured from the scheduled arrival, so a slow server cannot hide
    queueing) while the server runs in its own thread."""
    server.start()
    t0 = time.perf_counter()
    futs = []
    for req in requests:
        delay = t0 + req.arrival_s - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(req.frame, arrival=t0 + req.arrival_s))
    t_end = time.perf_counter() + drain_timeout
    while server.pending() and time.perf_counter() < t_end:
        time.sleep(0.001)
    server.stop()
    server.censor(time.perf_counter())
    return server.stats
