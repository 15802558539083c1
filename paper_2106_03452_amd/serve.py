"""Continuous-batching request engine for the Poisson solver.

Requests (an oriented point cloud, a resolution, and optionally dL/dchi for a
forward+backward solve) arrive at arbitrary times. The engine keeps resident
per-resolution slots (workspace, saved state, chi, gradients) carved out of an
HBM budget, admits waiting requests in arrival order as slots of their class
free up (later requests of another class may pass a blocked one), packs every
request admitted in one scheduling step into one ``psr_run_batched`` call, and
spreads those batches over several HIP streams so that their work overlaps on
the device. Completion is detected with events; arrival-to-completion latency
is recorded per request.

The scheduler is independent of the device: :class:`GpuBackend` drives the
library, :class:`MockBackend` is a timing model used to test admission,
ordering, back-pressure and error handling on the CPU.
"""
from __future__ import annotations

import collections
import ctypes
import heapq
import time
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    res: int
    npoints: int
    backward: bool
    arrival: float                      # host time (seconds) the request is due
    points: object = None               # device tensors (GpuBackend) or None (mock)
    normals: object = None
    dchi: object = None
    sigma: float = 2.0
    start: float | None = None          # time its batch was launched
    done: float | None = None           # completion time
    error: str | None = None
    slot: object = None
    out_chi: object = None              # optional caller tensors the results are copied into
    out_dpoints: object = None
    out_dnormals: object = None

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


@dataclass
class SlotClass:
    res: int
    max_points: int
    bytes_per_slot: int
    free: list = field(default_factory=list)
    total: int = 0


class Engine:
    """Admission + continuous batching over a backend.

    hbm_budget: bytes the resident slots may take in total.
    classes: {res: max_points} resolutions served and the largest point count per request.
    max_batch: most requests packed into one launch sequence.
    """

    def __init__(self, backend, classes: dict[int, int], hbm_budget: int, max_batch: int = 24,
                 max_inflight_per_stream: int = 2):
        self.backend = backend
        self.max_batch = max_batch
        self.max_inflight_per_stream = max_inflight_per_stream
        self.classes: dict[int, SlotClass] = {}
        per_class_budget = hbm_budget // max(1, len(classes))
        for res, pmax in sorted(classes.items()):
            b = backend.slot_bytes(res, pmax)
            self.classes[res] = SlotClass(res, pmax, b)
        # grow slots lazily up to the budget; a class always gets at least one slot
        self.budget = hbm_budget
        self.used = 0
        self.per_class_budget = per_class_budget
        self.waiting: collections.deque[Request] = collections.deque()
        self.inflight: list = []  # (handle, stream, [requests])
        self.finished: list[Request] = []
        self.rejected: list[Request] = []

    # ------------------------------------------------------------ admission
    def submit(self, req: Request) -> None:
        cls = self.classes.get(req.res)
        if cls is None or req.npoints > cls.max_points or req.npoints < 1:
            req.error = "rejected: resolution not served or point count out of range"
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _take_slot(self, cls: SlotClass):
        if cls.free:
            return cls.free.pop()
        fits = self.used + cls.bytes_per_slot <= self.budget
        fair = cls.total == 0 or cls.total * cls.bytes_per_slot + cls.bytes_per_slot <= self.per_class_budget
        if fits and fair:
            try:
                slot = self.backend.alloc_slot(cls.res, cls.max_points)
            except MemoryError:
                return None
            self.used += cls.bytes_per_slot
            cls.total += 1
            return slot
        return None

    def _admit(self) -> list[Request]:
        batch, kept = [], collections.deque()
        while self.waiting and len(batch) < self.max_batch:
            req = self.waiting.popleft()
            slot = self._take_slot(self.classes[req.res])
            if slot is None:
                kept.append(req)  # no slot of its class: stays queued, others may pass
                continue
            req.slot = slot
            batch.append(req)
        kept.extend(self.waiting)
        self.waiting = kept
        return batch

    # ------------------------------------------------------------ progress
    def _free_stream(self):
        busy = collections.Counter(s for _, s, _ in self.inflight)
        best = min(range(self.backend.num_streams), key=lambda s: busy[s])
        return best if busy[best] < self.max_inflight_per_stream else None

    def poll(self) -> int:
        """Retire completed batches; returns how many requests finished."""
        n = 0
        still = []
        for handle, stream, reqs in self.inflight:
            if self.backend.is_done(handle):
                t = self.backend.completion_time(handle)
                err = self.backend.error(handle)
                for r in reqs:
                    r.done = t
                    r.error = err
                    self.classes[r.res].free.append(r.slot)
                    r.slot = None
                    self.finished.append(r)
                n += len(reqs)
            else:
                still.append((handle, stream, reqs))
        self.inflight = still
        return n

    def step(self, now: float) -> int:
        """One scheduling step: retire, admit, launch. Returns requests launched."""
        self.poll()
        stream = self._free_stream()
        if stream is None or not self.waiting:
            return 0
        batch = self._admit()
        if not batch:
            return 0
        for r in batch:
            r.start = now
        handle = self.backend.launch(batch, stream)
        self.inflight.append((handle, stream, batch))
        return len(batch)

    def idle(self) -> bool:
        return not self.waiting and not self.inflight


def drive(engine: Engine, requests: list[Request], clock=time.perf_counter, spin_sleep: float = 0.0):
    """Feed `requests` (arrival times relative to the start) into the engine at
    their arrival times and run it until every request finished. Returns the
    start time used as the arrival origin."""
    t0 = clock()
    for r in requests:
        r.arrival += t0
    heap = [(r.arrival, r.rid, r) for r in requests]
    heapq.heapify(heap)
    while heap or not engine.idle():
        now = clock()
        while heap and heap[0][0] <= now:
            engine.submit(heapq.heappop(heap)[2])
        launched = engine.step(now)
        if not launched and spin_sleep:
            time.sleep(spin_sleep)
    return t0


def latency_stats(reqs: list[Request], skip: int = 0) -> dict:
    """p50/p99/mean of arrival-to-completion latency, skipping the `skip` earliest arrivals."""
    reqs = sorted(reqs, key=lambda r: r.arrival)
    lat = sorted(r.latency for r in reqs[skip:] if r.latency is not None)
    if not lat:
        return {}
    pick = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]
    return {"n": len(lat), "p50_ms": round(pick(0.50) * 1e3, 4), "p99_ms": round(pick(0.99) * 1e3, 4),
            "mean_ms": round(sum(lat) / len(lat) * 1e3, 4)}


# ---------------------------------------------------------------------------- backends
class MockBackend:
    """Timing model of the device for CPU tests: a batch takes
    sum(cost(res, backward)) / overlap seconds once launched; `fail_alloc`
    makes slot allocation fail after that many slots; `fail_launch` marks the
    given launch numbers as failed (their requests finish with an error)."""

    def __init__(self, num_streams=2, cost=None, clock=time.perf_counter, fail_alloc=None, fail_launch=()):
        self.num_streams = num_streams
        self.cost = cost or (lambda res, bwd: (res / 64.0) ** 3 * (2e-4 if bwd else 1e-4))
        self.clock = clock
        self.fail_alloc = fail_alloc
        self.fail_launch = set(fail_launch)
        self.allocated = 0
        self.launches = 0
        self.stream_free_at = [0.0] * num_streams

    def slot_bytes(self, res, pmax):
        return 12 * res ** 3 + 64 * pmax

    def alloc_slot(self, res, pmax):
        if self.fail_alloc is not None and self.allocated >= self.fail_alloc:
            raise MemoryError("mock allocation failure")
        self.allocated += 1
        return object()

    def launch(self, batch, stream):
        self.launches += 1
        now = self.clock()
        begin = max(now, self.stream_free_at[stream])
        end = begin + sum(self.cost(r.res, r.backward) for r in batch)
        self.stream_free_at[stream] = end
        return {"end": end, "failed": self.launches in self.fail_launch}

    def is_done(self, h):
        return self.clock() >= h["end"]

    def completion_time(self, h):
        return h["end"]

    def error(self, h):
        return "mock launch failure" if h["failed"] else None


class GpuBackend:
    """Drives libpsr: each batch is one psr_run_batched call on one of
    `num_streams` HIP streams; an event after it gives its completion time
    (GPU timestamps mapped onto the host clock through a reference event)."""

    def __init__(self, device=0, num_streams=4, sigma=2.0):
        import torch
        from . import _lib
        self.torch = torch
        self._lib = _lib
        self.dev = torch.device("cuda", device)
        self.ctx = _lib.context(device)
        self.num_streams = num_streams
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(num_streams)]
        self.sigma = sigma
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(torch.cuda.current_stream(self.dev))
        self.ref.synchronize()
        self.ref_host = time.perf_counter()

    def slot_bytes(self, res, pmax):
        L = self._lib
        return (L.workspace_bytes(res, pmax) + L.saved_bytes(res, pmax) + 4 * res ** 3 + 24 * pmax)

    def alloc_slot(self, res, pmax):
        torch = self.torch
        if hasattr(self, "ctx"):
            # the backward's point-source table of this size, built once now
            # rather than inside a batch
            self._lib.check(self._lib.lib().psr_ctx_prepare(
                self.ctx.handle, int(res), float(getattr(self, "sigma", 2.0)),
                ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)), "psr_ctx_prepare")
        try:
            return dict(
                ws=torch.empty(self._lib.workspace_bytes(res, pmax), dtype=torch.uint8, device=self.dev),
                saved=torch.empty(self._lib.saved_bytes(res, pmax), dtype=torch.uint8, device=self.dev),
                chi=torch.empty((res, res, res), dtype=torch.float32, device=self.dev),
                dp=torch.empty((pmax, 3), dtype=torch.float32, device=self.dev),
                dn=torch.empty((pmax, 3), dtype=torch.float32, device=self.dev))
        except RuntimeError as e:  # out of device memory
            raise MemoryError(str(e))

    def launch(self, batch, stream):
        torch = self.torch
        table = (self._lib.PsrJob * len(batch))()
        for e, r in zip(table, batch):
            s = r.slot
            e.points = r.points.data_ptr()
            e.normals = r.normals.data_ptr()
            e.npoints = r.npoints
            e.res = r.res
            e.sigma = r.sigma
            e.chi = s["chi"].data_ptr()
            e.saved = s["saved"].data_ptr()
            e.workspace = s["ws"].data_ptr()
            e.workspace_bytes = s["ws"].numel()
            if r.backward:
                e.dchi = r.dchi.data_ptr()
                e.dpoints = s["dp"].data_ptr()
                e.dnormals = s["dn"].data_ptr()
        st = self.streams[stream]
        # inputs were produced on the caller's stream: order after it
        st.wait_stream(torch.cuda.current_stream(self.dev))
        rc = self._lib.lib().psr_run_batched(self.ctx.handle, len(batch), table, ctypes.c_void_p(st.cuda_stream))
        if rc == 0:
            # deliver results before the completion event (the slot is reused afterwards)
            with torch.cuda.stream(st):
                for r in batch:
                    s = r.slot
                    if r.out_chi is not None:
                        r.out_chi.copy_(s["chi"], non_blocking=True)
                    if r.backward and r.out_dpoints is not None:
                        r.out_dpoints.copy_(s["dp"][: r.npoints], non_blocking=True)
                    if r.backward and r.out_dnormals is not None:
                        r.out_dnormals.copy_(s["dn"][: r.npoints], non_blocking=True)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        return {"ev": ev, "rc": rc, "table": table}

    def is_done(self, h):
        return h["rc"] != 0 or h["ev"].query()

    def completion_time(self, h):
        if h["rc"] != 0:
            return time.perf_counter()
        return self.ref_host + self.ref.elapsed_time(h["ev"]) * 1e-3

    def error(self, h):
        return None if h["rc"] == 0 else f"psr_run_batched failed: {self._lib.strerror(h['rc'])}"


class SequentialBaseline:
    """Plain solves one at a time on one stream in arrival order (no batching,
    no overlap): psr_forward then psr_backward per request."""

    def __init__(self, device=0):
        import torch
        from . import _lib
        self.torch = torch
        self._lib = _lib
        self.dev = torch.device("cuda", device)
        self.ctx = _lib.context(device)
        self.stream = torch.cuda.Stream(self.dev)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(torch.cuda.current_stream(self.dev))
        self.ref.synchronize()
        self.ref_host = time.perf_counter()
        self.slots = {}

    def _slot(self, res, pmax):
        if res not in self.slots:
            self.slots[res] = GpuBackend.alloc_slot(self, res, pmax)
        return self.slots[res]

    def run(self, requests, pmax_by_res, clock=time.perf_counter):
        torch, L = self.torch, self._lib.lib()
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        st = ctypes.c_void_p(self.stream.cuda_stream)
        t0 = clock()
        events = []
        for r in requests:
            r.arrival += t0
        for r in sorted(requests, key=lambda r: r.arrival):
            while clock() < r.arrival:
                pass
            s = self._slot(r.res, pmax_by_res[r.res])
            wsb = ctypes.c_size_t(s["ws"].numel())
            rc = L.psr_forward(self.ctx.handle, p(r.points), p(r.normals), r.npoints, r.res, r.sigma, p(s["chi"]),
                               p(s["saved"]), p(s["ws"]), wsb, st)
            if rc == 0 and r.backward:
                rc = L.psr_backward(self.ctx.handle, r.npoints, r.res, r.sigma, p(s["chi"]), p(s["saved"]),
                                    p(r.dchi), p(s["dp"]), p(s["dn"]), p(s["ws"]), wsb, st)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.stream)
            events.append((r, ev, rc))
        for r, ev, rc in events:
            ev.synchronize()
            r.done = self.ref_host + self.ref.elapsed_time(ev) * 1e-3
            r.error = None if rc == 0 else self._lib.strerror(rc)
        return t0
