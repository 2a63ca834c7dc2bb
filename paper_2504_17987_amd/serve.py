"""Batched graph launches and a continuous-batching server for streams of
image pairs.

The paper pipelines frames so that its fixed-function engine stays busy
while the compute units pre- and post-process neighbouring frames, and it
notes that small images are overhead-limited (Sec. 4.1).  Here the same
concern is met with batching and HIP graphs:

* ``GraphRunner`` captures the whole path (``piv_run``) into HIP graphs
  (``torch.cuda.CUDAGraph``), one per power-of-two bucket of slots up to its
  capacity; a device slot mask lets a replay run a partial bucket without
  recapture.
* ``Scheduler`` is the host policy of the server (pure Python, clock and
  executor injected, so it is tested on the CPU): stream admission against
  an HBM budget, per-size-class FIFO queues, launch when a class's slots
  are full, when its oldest request has waited ``max_wait``, when the
  device is idle or when the class has nothing on the device; up to
  ``inflight`` batches per class on the device.
* ``GpuExecutor`` runs a class's batch as one graph replay on that class's
  own stream (classes overlap on the device) and polls HIP events for
  completion.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

# ----------------------------------------------------------------------------
# graph runner (device)
# ----------------------------------------------------------------------------


class GraphRunner:
    """Static slot buffers + captured graphs of the whole path.

    One graph per bucket size (1, 2, 4, ... up to ``slots``), each over the
    first n slots, so that a partial batch launches grids for the smallest
    bucket that holds it instead of the full capacity; the device slot mask
    switches off the bucket's unused slots.  The plan must be dedicated to
    this runner (its workspace and slot mask are used by the captured
    kernels), with max_batch >= slots."""

    def __init__(self, plan, slots: int, stream=None, temporal: Optional[dict] = None):
        """temporal (optional): dict(state_pred=, state_disp=, alpha1=,
        alpha2=) -- the captured path is then piv_run_temporal with this
        runner's device slot table (``set_slots``) into those states."""
        import torch
        from .api import Plan  # noqa: F401
        self.torch = torch
        self.plan = plan
        self.slots = slots
        self.temporal = temporal
        dev = plan.device
        H, W = plan.height, plan.width
        self.A = torch.zeros((slots, H, W), dtype=plan.tdtype, device=dev)
        self.B = torch.zeros((slots, H, W), dtype=plan.tdtype, device=dev)
        ny, nx = plan.ny, plan.nx
        self.out = dict(pred=torch.zeros((slots, 2, ny, nx), device=dev),
                        disp=torch.zeros((slots, 2, ny, nx), device=dev),
                        peak=torch.zeros((slots, ny, nx), device=dev),
                        flags=torch.zeros((slots, ny, nx), dtype=torch.uint8, device=dev),
                        omega=torch.zeros((slots, ny, nx), device=dev))
        self.mask = torch.ones((slots,), dtype=torch.uint8, device=dev)
        # smoothing state slot of each batch slot (device), written from a
        # pinned host copy before each launch (see set_slots)
        self.slot = torch.zeros((slots,), dtype=torch.int32, device=dev)
        self.slot_host = torch.zeros((slots,), dtype=torch.int32, pin_memory=True) if temporal else None
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        b, self.buckets = 1, []
        while b < slots:
            self.buckets.append(b)
            b *= 2
        self.buckets.append(slots)
        self.graphs: Dict[int, object] = {}
        self._mask_state: Optional[Tuple[int, int]] = None   # (active, upto) last written

    @property
    def graph(self):
        return self.graphs.get(self.slots)

    def resident_bytes(self) -> int:
        t = [self.A, self.B, self.mask, self.slot] + list(self.out.values())
        return sum(x.numel() * x.element_size() for x in t) + self.plan.workspace_bytes(self.slots)

    @staticmethod
    def bytes_for(plan, slots: int) -> int:
        """resident_bytes() of a runner of `slots` slots on `plan`'s geometry,
        computed before any device memory is allocated."""
        es = {"u8": 1, "u16": 2, "f32": 4}[plan.dtype]
        npx = plan.ny * plan.nx
        per = 2 * plan.width * plan.height * es + 4 * (2 + 2 + 1 + 1) * npx + npx + 1 + 4
        return slots * per + plan.workspace_bytes(slots)

    def path(self, A, B, out, n: int) -> None:
        """One call of the path on the first n slots (the captured call)."""
        t = self.temporal
        if t is None:
            self.plan.run(A, B, out)
        else:
            self.plan.run_temporal(A, B, self.slot[:n], t.get("state_pred"), t.get("state_disp"),
                                   t.get("alpha1", 0.5), t.get("alpha2", 0.5), out)

    def set_slots(self, slots: Sequence[int]) -> None:
        """Write the smoothing state slot of batch slots 0..len-1 (k continues
        state k, -1 - k starts it), on the runner's stream.  The pinned host
        copy is reused, which is safe because a runner holds at most one live
        batch: the previous copy from it completed before this runner was
        handed out again."""
        if self.slot_host is None:
            raise RuntimeError("runner was built without temporal smoothing")
        k = len(slots)
        self.slot_host[:k] = self.torch.tensor(list(slots), dtype=self.torch.int32)
        with self.torch.cuda.stream(self.stream):
            self.slot[:k].copy_(self.slot_host[:k], non_blocking=True)

    def bucket(self, n: int) -> int:
        return next(b for b in self.buckets if b >= n)

    def capture(self) -> None:
        torch = self.torch
        self.plan.bind_slot_mask(self.mask)
        self._mask_state = None
        self.stream.wait_stream(torch.cuda.current_stream())
        for n in self.buckets:
            A, B = self.A[:n], self.B[:n]
            out = {k: v[:n] for k, v in self.out.items()}
            # warm up on the capture stream, then capture (with smoothing on,
            # the warm-up runs with every slot outside the state tables, so
            # no state is touched)
            if self.temporal is not None:
                with torch.cuda.stream(self.stream):
                    self.slot.fill_(-(1 << 30))
            with torch.cuda.stream(self.stream):
                self.path(A, B, out, n)
            self.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self.path(A, B, out, n)
            self.stream.synchronize()
            self.graphs[n] = g

    def set_active(self, n: int, upto: Optional[int] = None) -> None:
        """Slots [0, n) run, slots [n, upto) are skipped (small fill kernels
        on the runner's stream; no memset node).  Skipped when the mask
        already reads so."""
        upto = self.slots if upto is None else upto
        st = self._mask_state
        if st is not None and st[0] == n and (n >= upto or st[1] >= upto):
            return
        with self.torch.cuda.stream(self.stream):
            self.mask[:n].fill_(1)
            if n < upto:
                self.mask[n:upto].fill_(0)
        self._mask_state = (n, upto)

    def replay(self, n: Optional[int] = None) -> None:
        """Replay the graph of the smallest bucket holding n slots (all slots
        when n is None), after all work already queued on the caller's
        current stream (input copies, for instance)."""
        if not self.graphs:
            self.capture()
        self.stream.wait_stream(self.torch.cuda.current_stream())
        b = self.slots if n is None else self.bucket(n)
        self.set_active(self.slots if n is None else n, b)
        with self.torch.cuda.stream(self.stream):
            self.graphs[b].replay()


# ----------------------------------------------------------------------------
# host policy (CPU-testable)
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class Request:
    rid: int
    stream: int
    cls: str
    item: int            # which of the stream's resident pairs
    arrival: float
    start: float = math.nan
    done: float = math.nan


@dataclasses.dataclass
class ClassSpec:
    name: str
    width: int
    height: int
    capacity: int        # slots per batch
    slot_bytes: int      # resident bytes of one runner (plan workspace, slots, outputs)
    stream_bytes: int    # resident bytes of one admitted stream (its device-resident pairs)


class Executor:
    """What the scheduler needs from the device side."""

    def launch(self, cls: str, reqs: List[Request], now: float) -> object: ...

    def done(self, handle: object) -> bool: ...

    def busy(self) -> bool: ...

    def class_admitted(self, cls: str) -> None:
        """The first stream of `cls` was admitted: build its runners."""

    def class_retired(self, cls: str) -> None:
        """The last stream of `cls` retired and none of its batches runs:
        release its runners."""


class Scheduler:
    """Continuous batching over size classes.

    * admit(stream, cls): reserves the class's runners (first stream of a
      class) and the stream's resident bytes against ``budget``; a stream
      that does not fit waits in the admission queue and is admitted as
      soon as memory is released (``retire``).
    * submit(req): requests of admitted streams join their class's FIFO.
    * step(now): completes finished batches, then launches, per class and
      while that class has fewer than ``inflight`` batches on the device,
      the oldest ``capacity`` requests when the queue is full, when the
      oldest has waited ``max_wait``, when the device is idle, or when the
      class has no batch on the device (so light load never waits and heavy
      load batches by itself).
    """

    def __init__(self, classes: Sequence[ClassSpec], executor: Executor, budget: int,
                 max_wait: float = 2e-3, inflight: int = 2):
        self.classes = {c.name: c for c in classes}
        self.ex = executor
        self.budget = budget
        self.max_wait = max_wait
        self.inflight = inflight
        self.used = 0
        self.admitted: Dict[int, str] = {}
        self.waiting: Deque[Tuple[int, str]] = collections.deque()
        self.class_live: Dict[str, int] = collections.Counter()
        self.queues: Dict[str, Deque[Request]] = {c: collections.deque() for c in self.classes}
        self.running: Dict[str, List[Tuple[object, List[Request]]]] = {c: [] for c in self.classes}
        self.finished: List[Request] = []
        self.refused: List[Request] = []   # requests of streams not admitted (or retired)
        self.refused_submits = 0
        self.batches = 0
        self._release_after: set = set()

    # -- admission ----------------------------------------------------------
    def _cost(self, cls: str) -> int:
        c = self.classes[cls]
        cost = c.stream_bytes
        if self.class_live[cls] == 0:
            cost += self.inflight * c.slot_bytes
        return cost

    def _try_admit(self, stream: int, cls: str) -> bool:
        if self.used + self._cost(cls) <= self.budget:
            self.used += self._cost(cls)
            first = self.class_live[cls] == 0
            self.class_live[cls] += 1
            self.admitted[stream] = cls
            if first:
                # the class's runners are charged to the budget now and
                # built now, so the ledger governs real memory
                self.ex.class_admitted(cls)
            return True
        return False

    def admit(self, stream: int, cls: str) -> bool:
        if stream in self.admitted:
            return True
        if self._try_admit(stream, cls):
            return True
        if (stream, cls) not in self.waiting:
            self.waiting.append((stream, cls))
        return False

    def retire(self, stream: int) -> None:
        """Retire an admitted stream; its queued requests are dropped (and
        counted as refused).  The class's runners are released with its last
        stream, once none of its batches is on the device."""
        cls = self.admitted.pop(stream, None)
        if cls is not None:
            q = self.queues[cls]
            keep = collections.deque(r for r in q if r.stream != stream)
            self.refused.extend(r for r in q if r.stream == stream)
            self.queues[cls] = keep
            self.class_live[cls] -= 1
            self.used -= self.classes[cls].stream_bytes
            if self.class_live[cls] == 0:
                self.used -= self.inflight * self.classes[cls].slot_bytes
                if self.running[cls]:
                    self._release_after.add(cls)
                else:
                    self.ex.class_retired(cls)
        self._drain_waiting()

    def set_budget(self, budget: int) -> None:
        self.budget = budget
        self._drain_waiting()

    def _drain_waiting(self) -> None:
        # admit waiting streams in order while they fit
        still = collections.deque()
        while self.waiting:
            s, c = self.waiting.popleft()
            if not self._try_admit(s, c):
                still.append((s, c))
        self.waiting = still

    # -- requests -----------------------------------------------------------
    def submit(self, req: Request) -> bool:
        if self.admitted.get(req.stream) != req.cls:
            self.refused_submits += 1
            self.refused.append(req)
            return False
        self.queues[req.cls].append(req)
        return True

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values()) + sum(
            sum(len(r) for _, r in v) for v in self.running.values())

    def step(self, now: float) -> int:
        """One scheduling round; returns the number of batches launched."""
        for cls, lst in self.running.items():
            keep = []
            for h, reqs in lst:
                if self.ex.done(h):
                    for r in reqs:
                        r.done = now
                    self.finished.extend(reqs)
                else:
                    keep.append((h, reqs))
            self.running[cls] = keep
            if cls in self._release_after and not keep and self.class_live[cls] == 0:
                self._release_after.discard(cls)
                self.ex.class_retired(cls)
        launched = 0
        idle = not self.ex.busy()
        # oldest-first across classes so that no class starves
        order = sorted((q[0].arrival, cls) for cls, q in self.queues.items() if q)
        for _, cls in order:
            q = self.queues[cls]
            cap = self.classes[cls].capacity
            while q and len(self.running[cls]) < self.inflight:
                full = len(q) >= cap
                late = now - q[0].arrival >= self.max_wait
                # a class with nothing on the device launches at once: its
                # requests never wait behind another class's batch
                cls_idle = not self.running[cls]
                if not (full or late or idle or cls_idle):
                    break
                batch = [q.popleft() for _ in range(min(cap, len(q)))]
                for r in batch:
                    r.start = now
                h = self.ex.launch(cls, batch, now)
                self.running[cls].append((h, batch))
                self.batches += 1
                launched += 1
                idle = False
        return launched


class FakeExecutor(Executor):
    """Scripted batch durations on a simulated clock (CPU tests)."""

    def __init__(self, duration: Callable[[str, int], float], clock: Callable[[], float]):
        self.duration = duration
        self.clock = clock
        self.live: Dict[int, float] = {}
        self.n = 0
        self.log: List[Tuple[str, int, float]] = []

    def launch(self, cls, reqs, now):
        self.n += 1
        self.live[self.n] = now + self.duration(cls, len(reqs))
        self.log.append((cls, len(reqs), now))
        return self.n

    def done(self, h):
        if self.live[h] <= self.clock():
            del self.live[h]
            return True
        return False

    def busy(self):
        t = self.clock()
        return any(v > t for v in self.live.values())


# ----------------------------------------------------------------------------
# device executor and the server loop
# ----------------------------------------------------------------------------


class GpuExecutor(Executor):
    """Graph replays on per-class streams; completion by HIP events.

    A class's runners (``inflight`` of them, each with its own plan,
    workspace, HIP stream and captured graphs) are built when the class's
    first stream is admitted and released when its last stream retires.
    ``pairs[stream]`` holds each admitted stream's device-resident pairs
    (A, B tensors of shape [k, H, W]); a launch copies the requested pairs
    into a free runner's slots (device-to-device, on the runner's stream),
    sets the active-slot mask and replays the runner's graph.  A batch of
    one pair (what light load produces) skips the copies and the graph: the
    runner's plan runs that pair eagerly from its own buffers into slot 0
    (same kernels, same workspace, same stream).  The pairs must be written
    (complete on the device) before the first launch that reads them:
    launches do not order themselves after other streams.  Each runner has
    one completion event, reused, since it holds at most one live batch.

    With ``temporal`` (dict(alpha1=, alpha2=)) each class keeps resident
    smoothing states for its streams and runs the paper's path with
    exponential smoothing in time (piv_run_temporal): a stream's first
    request starts its state, later ones continue it.  Results then depend
    on each stream's history, so the launches of one class are ordered on
    the device (each waits for the class's previous launch)."""

    def __init__(self, classes: Dict[str, Tuple[int, int, int]], pairs: Dict[int, Tuple[object, object]],
                 stream_class: Dict[int, str], plan_kw: Optional[dict] = None, inflight: int = 2,
                 keep_results: bool = False, eager_single: bool = True, temporal: Optional[dict] = None):
        import torch
        self.torch = torch
        self.classes = classes
        self.pairs = pairs
        self.stream_class = stream_class
        self.plan_kw = dict(plan_kw or {})
        self.inflight = inflight
        self.runners: Dict[str, List[GraphRunner]] = {}
        self.free: Dict[str, List[GraphRunner]] = {}
        self.live: Dict[int, Tuple[str, GraphRunner, object, List[Request]]] = {}
        self.n = 0
        self.keep = keep_results
        self.eager_single = eager_single
        self.results: Dict[int, Dict[str, object]] = {}
        self.slot0: Dict[int, Dict[str, object]] = {}
        self.event: Dict[int, object] = {}
        self.temporal = temporal
        self.state_index: Dict[int, int] = {}
        for c in classes:
            for k, s in enumerate(sorted(s for s, cc in stream_class.items() if cc == c)):
                self.state_index[s] = k
        self.started: set = set()
        self.states: Dict[str, Dict[str, object]] = {}
        self.last_event: Dict[str, object] = {}
        self.batch_sizes: List[int] = []   # size of every launched batch, in launch order

    def runner_bytes(self, cls: str) -> int:
        from .api import Plan
        W, H, cap = self.classes[cls]
        p = Plan(W, H, max_batch=cap, workspace=False, **self.plan_kw)
        b = GraphRunner.bytes_for(p, cap)
        if self.temporal is not None:
            # the class's two smoothing state tables, shared by its runners
            # (the scheduler charges runner_bytes once per runner)
            nst = sum(1 for c in self.stream_class.values() if c == cls)
            b += -(-2 * 4 * nst * 2 * p.ny * p.nx // self.inflight)
        p.close()
        return b

    def class_admitted(self, cls: str) -> None:
        if cls in self.runners:
            return
        torch = self.torch
        from .api import Plan
        W, H, cap = self.classes[cls]
        tm = None
        if self.temporal is not None:
            nst = sum(1 for c in self.stream_class.values() if c == cls)
            probe = Plan(W, H, max_batch=cap, workspace=False, **self.plan_kw)
            st = dict(state_pred=probe.new_state(nst), state_disp=probe.new_state(nst))
            probe.close()
            self.states[cls] = st
            tm = dict(st, alpha1=self.temporal.get("alpha1", 0.5), alpha2=self.temporal.get("alpha2", 0.5))
        rs = []
        for _ in range(self.inflight):
            r = GraphRunner(Plan(W, H, max_batch=cap, **self.plan_kw), cap, temporal=tm)
            r.capture()
            rs.append(r)
        # the runners' buffers and graphs are complete before their first launch
        torch.cuda.synchronize()
        self.runners[cls] = rs
        self.free[cls] = list(rs)
        for r in rs:
            self.slot0[id(r)] = {k: v[0:1] for k, v in r.out.items()}
            self.event[id(r)] = torch.cuda.Event()

    def class_retired(self, cls: str) -> None:
        for r in self.runners.pop(cls, []):
            self.slot0.pop(id(r), None)
            self.event.pop(id(r), None)
        self.free.pop(cls, None)
        self.states.pop(cls, None)
        self.last_event.pop(cls, None)
        self.started = {s for s in self.started if self.stream_class.get(s) != cls}

    def _slot_values(self, reqs: List[Request]) -> List[int]:
        vals = []
        for r in reqs:
            k = self.state_index[r.stream]
            if r.stream in self.started:
                vals.append(k)
            else:
                vals.append(-1 - k)
                self.started.add(r.stream)
        return vals

    def launch(self, cls, reqs, now):
        torch = self.torch
        run = self.free[cls].pop()
        self.batch_sizes.append(len(reqs))
        if self.temporal is not None:
            run.set_slots(self._slot_values(reqs))
            prev = self.last_event.get(cls)
            if prev is not None:
                run.stream.wait_event(prev)
        if len(reqs) == 1 and self.eager_single:
            r = reqs[0]
            a, b = self.pairs[r.stream]
            # (the plan's slot mask is the runner's; slot 0 is active under
            # every mask set_active writes, and the mask starts all ones)
            with torch.cuda.stream(run.stream):
                run.path(a[r.item:r.item + 1], b[r.item:r.item + 1], self.slot0[id(run)], 1)
        else:
            with torch.cuda.stream(run.stream):
                for i, r in enumerate(reqs):
                    a, b = self.pairs[r.stream]
                    run.A[i].copy_(a[r.item], non_blocking=True)
                    run.B[i].copy_(b[r.item], non_blocking=True)
            run.replay(len(reqs))
        ev = self.event[id(run)]
        ev.record(run.stream)
        if self.temporal is not None:
            self.last_event[cls] = ev
        self.n += 1
        self.live[self.n] = (cls, run, ev, reqs)
        return self.n

    def done(self, h):
        cls, run, ev, reqs = self.live[h]
        if not ev.query():
            return False
        torch = self.torch
        if self.keep:
            # the copies run on the runner's stream, so its next launch (which
            # rewrites the slots) is ordered after them; the caller's stream
            # waits for them before it reads the results
            with torch.cuda.stream(run.stream):
                for i, r in enumerate(reqs):
                    self.results[r.rid] = {k: v[i].clone() for k, v in run.out.items()}
            torch.cuda.current_stream().wait_stream(run.stream)
        del self.live[h]
        self.free[cls].append(run)
        return True

    def busy(self):
        return bool(self.live)


def make_gpu_server(classes: Dict[str, Tuple[int, int, int]], pairs: Dict[int, Tuple[object, object]],
                    stream_class: Dict[int, str], budget: int, plan_kw: Optional[dict] = None,
                    inflight: int = 2, max_wait: float = 2e-3, keep_results: bool = False,
                    eager_single: bool = True, temporal: Optional[dict] = None):
    """Build the executor and the scheduler and admit the streams in order;
    a class's runners (``inflight`` per class) are built when its first
    stream is admitted.  classes: name -> (W, H, slots).  Returns
    (scheduler, executor)."""
    import torch
    ex = GpuExecutor(classes, pairs, stream_class, plan_kw=plan_kw, inflight=inflight,
                     keep_results=keep_results, eager_single=eager_single, temporal=temporal)
    specs = []
    for name, (W, H, cap) in classes.items():
        per_stream = 0
        for s, c in stream_class.items():
            if c == name:
                a, b = pairs[s]
                per_stream = a.numel() * a.element_size() + b.numel() * b.element_size()
                break
        specs.append(ClassSpec(name, W, H, cap, ex.runner_bytes(name), per_stream))
    # the admitted pairs are complete before the first launch reads them
    torch.cuda.synchronize()
    sched = Scheduler(specs, ex, budget, max_wait=max_wait, inflight=inflight)
    for s, c in stream_class.items():
        sched.admit(s, c)
    return sched, ex


def poisson_trace(streams: Sequence[Tuple[int, str]], rate: float, duration: float, items: int,
                  seed: int = 0) -> List[Request]:
    """Merged Poisson arrivals: each stream at `rate` requests/s for
    `duration` seconds, cycling through its `items` resident pairs."""
    import numpy as np
    rng = np.random.default_rng(seed)
    reqs = []
    for s, cls in streams:
        t, k = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration:
                break
            reqs.append(Request(0, s, cls, k % items, t))
            k += 1
    reqs.sort(key=lambda r: (r.arrival, r.stream))
    for i, r in enumerate(reqs):
        r.rid = i
    return reqs


def serve_trace(sched: Scheduler, trace: List[Request], clock: Callable[[], float],
                poll: float = 20e-6, deadline: float = 60.0) -> List[Request]:
    """Feed `trace` (arrival times relative to the start) into `sched` in
    real time and run until every accepted request has completed.  Returns
    the requests refused (their streams were not admitted); those keep a
    NaN completion time and stay out of ``latency_stats``."""
    n_ref = len(sched.refused)
    t0 = clock()
    i = 0
    while i < len(trace) or sched.pending():
        now = clock() - t0
        if now > deadline:
            raise TimeoutError(f"serving did not finish within {deadline} s")
        while i < len(trace) and trace[i].arrival <= now:
            sched.submit(trace[i])
            i += 1
        if not sched.step(now) and poll > 0:
            time.sleep(poll)
    return sched.refused[n_ref:]


def run_fifo(plan_for: Callable[[str], object], pairs, trace: List[Request], clock,
             deadline: float = 120.0) -> None:
    """The plain per-pair form: one request at a time in arrival order, each
    an ordinary (non-graph) piv_run of one pair; completion synchronously."""
    import torch
    t0 = clock()
    for r in trace:
        while clock() - t0 < r.arrival:
            pass
        r.start = clock() - t0
        a, b = pairs[r.stream]
        plan = plan_for(r.cls)
        plan.run(a[r.item:r.item + 1], b[r.item:r.item + 1], plan._fifo_out)
        torch.cuda.current_stream().synchronize()
        r.done = clock() - t0
        if r.done > deadline:
            raise TimeoutError("FIFO baseline exceeded its deadline")


def latency_stats(reqs: Sequence[Request]) -> Dict[str, float]:
    """Latency percentiles and throughput of the completed requests (refused
    ones, with a NaN completion time, are counted apart)."""
    import numpy as np
    done = [r for r in reqs if not math.isnan(r.done)]
    refused = len(reqs) - len(done)
    if not done:
        return {"p50_ms": math.nan, "p99_ms": math.nan, "mean_ms": math.nan, "pairs_per_s": 0.0, "n": 0,
                "refused": refused}
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "pairs_per_s": len(done) / span if span > 0 else math.nan,
            "n": len(done), "refused": refused}
