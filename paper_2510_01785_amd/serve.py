"""Serving loop: continuous batching of mixed (nside, lmax) transform requests
on one GPU, with admission against an HBM budget and overlap on streams.

A request is one map2alm or alm2map call on a batch of channels already
resident in device memory.  `Server.submit` queues it and returns a Future.
An admission thread scans the queue in arrival order and starts the first
request whose device memory (output and workspace, plus the resident tables
of an (nside, lmax) not seen before) fits in what is left of the budget, when
a stream slot is free: a large request at the head that does not fit yet does
not hold back smaller ones behind it, but once it has been passed over
`max_skips` times nothing behind it is admitted until it has started (no
starvation).  Queued requests of the same geometry (direction, nside, lmax, dtype) are
merged with the admitted one into a single transform call on the
concatenated channels, up to `max_merge_channels` channels and as far as the
budget allows: one launch of B channels runs the matrix-core kernels and
costs much less per map than several small ones, and each request receives
its own slice of the result.  A request runs on its slot's stream and an
event marks its end.
A completion thread resolves the futures in completion order, then returns
the request's transient memory and its slot, which admits the next requests.
Tables stay resident once built, so their bytes stay charged to the budget.

* A request whose memory alone exceeds the budget is rejected at submit
  (its future fails with `AdmissionError`); nothing is allocated.
* A queued request can be cancelled (Future.cancel) or time out in the queue;
  it is dropped without touching the GPU.
* Per request the loop records arrival, admit and done times; `stats()`
  reports p50/p99 latency, maps/s, memory in use and queue depth.
* The budget covers what the loop allocates while a request runs (output,
  workspace) and the tables it keeps resident; a finished request's output
  belongs to its future, i.e. to the caller.

The scheduling core (`Scheduler`) is independent of the device: it drives an
executor with `need(req)` (bytes held while the request runs, or a pair
(those bytes, bytes that stay resident once it has run)), `launch(req,
slot)`, `done(handle)` and `finish(handle)`; an executor that also offers
`group_key(req)`, `need_group(reqs)` and `launch_group(reqs, slot)` (whose
`finish` returns one result per request) gets merged requests.  `Server` pairs it with the GPU executor built on the C-ABI
binding (`ops`); tests drive it with a host executor.
"""
import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass, field

import numpy as np


class AdmissionError(RuntimeError):
    """The request needs more device memory than the whole budget."""


@dataclass
class Request:
    direction: str          # "map2alm" or "alm2map"
    nside: int
    lmax: int
    data: object            # device tensor: maps [B, Npix] or alm [B, nalm]
    timeout: float = None   # seconds the request may wait in the queue
    # filled in by the scheduler (seconds, time.perf_counter)
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    need: int = 0           # bytes returned to the budget when the request ends
    skipped: int = 0        # times a later request was admitted ahead of this one
    future: concurrent.futures.Future = field(default_factory=concurrent.futures.Future)

    @property
    def batch(self):
        return int(self.data.shape[0]) if getattr(self.data, "dim", lambda: 1)() > 1 else 1


@dataclass
class Done:
    t_arrival: float
    t_admit: float
    t_done: float
    batch: int
    need: int


def _split_need(n):
    """(transient, resident) bytes from an executor's need()."""
    if isinstance(n, tuple):
        return int(n[0]), int(n[1])
    return int(n), 0


class Scheduler:
    """Admission under a memory budget and a slot count: arrival order, with
    requests that fit admitted ahead of a blocked head at most `max_skips`
    times (default: twice the slot count)."""

    def __init__(self, executor, budget_bytes, slots, poll_s=2e-4, max_skips=None, max_merge_channels=0):
        self.ex = executor
        # merging needs the executor's group interface
        self.max_merge = int(max_merge_channels) if hasattr(executor, "launch_group") else 0
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.poll_s = poll_s
        self.max_skips = 2 * self.slots if max_skips is None else int(max_skips)
        self.resident = 0            # bytes that stay charged (tables kept resident)
        self._cv = threading.Condition()
        self._queue = collections.deque()
        self._free_slots = list(range(self.slots))
        self._running = {}           # slot -> (request, handle)
        self._launching = 0          # admitted, launch in progress
        self.in_use = 0
        self.peak_in_use = 0
        self.launches = 0            # transform calls (a merged job is one)
        self.finished = []
        self._closed = False
        self._threads = [threading.Thread(target=self._admit_loop, daemon=True),
                         threading.Thread(target=self._complete_loop, daemon=True)]
        for t in self._threads:
            t.start()

    # ---------------------------------------------------------------- API
    def submit(self, req):
        req.t_arrival = time.perf_counter()
        t, r = _split_need(self.ex.need(req))
        if t + r > self.budget - self.resident:
            req.future.set_exception(AdmissionError(
                "request needs %d bytes, budget is %d (%d held by resident tables)"
                % (t + r, self.budget, self.resident)))
            return req.future
        with self._cv:
            if self._closed:
                raise RuntimeError("scheduler closed")
            self._queue.append(req)
            self._cv.notify_all()
        return req.future

    def queue_depth(self):
        with self._cv:
            return len(self._queue)

    def drain(self):
        """Block until nothing is queued or running."""
        with self._cv:
            while self._queue or self._running or self._launching:
                self._cv.wait(0.05)

    def close(self):
        self.drain()
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    # ----------------------------------------------------------- threads
    def _pick_locked(self):
        """Queue indices of the job to admit now (the first queued request
        that fits, scanning no further than a request that has been passed
        over max_skips times, plus the queued requests merged with it) and
        its (transient, resident) bytes, or None."""
        if not self._free_slots:
            return None
        for i, r in enumerate(self._queue):
            t, res = _split_need(self.ex.need(r))
            if self.in_use + t + res <= self.budget:
                return self._merge_locked(i, t, res)
            if r.skipped >= self.max_skips:
                return None
        return None

    def _merge_locked(self, i, t, res):
        """Request i and the later queued requests of its group key that fit
        (channels up to max_merge_channels, bytes within the budget)."""
        idx = [i]
        if self.max_merge <= 0:
            return idx, t, res
        head = self._queue[i]
        key = self.ex.group_key(head)
        chans = head.batch
        for j in range(i + 1, len(self._queue)):
            r = self._queue[j]
            if r.future.cancelled() or self.ex.group_key(r) != key or chans + r.batch > self.max_merge:
                continue
            tj, rj = _split_need(self.ex.need_group([self._queue[k] for k in idx] + [r]))
            if self.in_use + tj + rj <= self.budget:
                idx.append(j)
                chans += r.batch
                t, res = tj, rj
        return idx, t, res

    def _admit_loop(self):
        while True:
            with self._cv:
                while True:
                    if self._closed and not self._queue:
                        return
                    self._drop_dead_locked()
                    pick = self._pick_locked()
                    if pick is not None:
                        break
                    self._cv.wait(0.05)
                idx, t, res = pick
                job = [self._queue[k] for k in idx]
                for k in sorted(idx, reverse=True):
                    del self._queue[k]
                for j in range(idx[0]):
                    self._queue[j].skipped += 1
                job = [r for r in job if r.future.set_running_or_notify_cancel()]
                if not job:
                    continue
                if len(job) < len(idx):  # a request was cancelled meanwhile: recount its job
                    t, res = _split_need(self.ex.need_group(job) if len(job) > 1 else self.ex.need(job[0]))
                slot = self._free_slots.pop(0)
                job[0].need = t  # the job's transient bytes, returned when it ends
                self.in_use += t + res
                self.resident += res
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                now = time.perf_counter()
                for r in job:
                    r.t_admit = now
                self._launching += 1
            try:
                handle = self.ex.launch_group(job, slot) if len(job) > 1 else self.ex.launch(job[0], slot)
            except Exception as e:  # launch failed: release and report
                # resident bytes go back too if the tables were not kept
                lost = res if _split_need(self.ex.need(job[0]))[1] > 0 else 0
                with self._cv:
                    self.in_use -= job[0].need + lost
                    self.resident -= lost
                    self._free_slots.append(slot)
                    self._launching -= 1
                    self._cv.notify_all()
                for r in job:
                    r.future.set_exception(e)
                continue
            with self._cv:
                self._running[slot] = (job, handle)
                self.launches += 1
                self._launching -= 1
                self._cv.notify_all()

    def _drop_dead_locked(self):
        """Cancelled or timed-out requests leave the queue untouched by the GPU."""
        now = time.perf_counter()
        keep = collections.deque()
        for r in self._queue:
            if r.future.cancelled():
                continue
            if r.timeout is not None and now - r.t_arrival > r.timeout:
                r.future.set_exception(TimeoutError("request timed out in the queue"))
                continue
            keep.append(r)
        self._queue = keep

    def _complete_loop(self):
        while True:
            with self._cv:
                if self._closed and not self._running and not self._queue and not self._launching:
                    return
                running = list(self._running.items())
            done_any = False
            for slot, (job, handle) in running:
                if not self.ex.done(handle):
                    continue
                try:
                    result = self.ex.finish(handle)
                    results = result if len(job) > 1 else [result]
                    err = None
                except Exception as e:
                    results, err = None, e
                now = time.perf_counter()
                with self._cv:
                    del self._running[slot]
                    self.in_use -= job[0].need
                    self._free_slots.append(slot)
                    # timing records only: the results stay with the callers' futures
                    for r in job:
                        r.t_done = now
                        self.finished.append(Done(r.t_arrival, r.t_admit, r.t_done, r.batch,
                                                  job[0].need if r is job[0] else 0))
                    self._cv.notify_all()
                for k, r in enumerate(job):
                    if err is None:
                        r.future.set_result(results[k])
                    else:
                        r.future.set_exception(err)
                done_any = True
            if not done_any:
                time.sleep(self.poll_s)

    # -------------------------------------------------------------- stats
    def stats(self, t0=None, t1=None):
        with self._cv:
            fin = list(self.finished)
            depth = len(self._queue)
            in_use = self.in_use
            resident = self.resident
        if not fin:
            return dict(requests=0, queue_depth=depth, in_use_bytes=in_use, resident_bytes=resident,
                        peak_in_use_bytes=self.peak_in_use)
        lat = np.array([r.t_done - r.t_arrival for r in fin]) * 1e3
        wait = np.array([r.t_admit - r.t_arrival for r in fin]) * 1e3
        t0 = min(r.t_arrival for r in fin) if t0 is None else t0
        t1 = max(r.t_done for r in fin) if t1 is None else t1
        maps = sum(r.batch for r in fin)
        return dict(requests=len(fin), launches=self.launches, maps=maps, maps_per_s=maps / max(t1 - t0, 1e-12),
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    queue_wait_p50_ms=float(np.percentile(wait, 50)),
                    queue_wait_p99_ms=float(np.percentile(wait, 99)),
                    queue_depth=depth, in_use_bytes=in_use, resident_bytes=resident,
                    peak_in_use_bytes=self.peak_in_use, budget_bytes=self.budget)


class GpuExecutor:
    """Runs requests through the library on per-slot HIP streams."""

    def __init__(self, device, slots):
        import torch
        from . import ops
        self.torch, self.ops = torch, ops
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]  # default priority
        self.table_stream = torch.cuda.Stream(device=self.device)  # default priority
        self._tables_lock = threading.Lock()
        self._tables = {}  # (nside, lmax) -> event recorded after the tables' build

    def _out_bytes(self, req):
        B = req.batch
        if req.direction == "map2alm":
            csize = 16 if req.data.dtype == self.torch.float64 else 8
            return B * self.ops.nalm(req.lmax) * csize
        esize = 8 if req.data.dtype == self.torch.complex128 else 4
        return B * self.ops.npix(req.nside) * esize

    def _code(self, req):
        from . import _lib
        if req.direction == "map2alm":
            return {self.torch.float64: _lib.F64, self.torch.float32: _lib.F32,
                    self.torch.bfloat16: _lib.BF16}[req.data.dtype]
        if req.direction == "alm2map":
            return {self.torch.complex128: _lib.F64, self.torch.complex64: _lib.F32}[req.data.dtype]
        raise ValueError("unknown direction %r" % req.direction)

    def need(self, req):
        return self.need_group([req])

    def group_key(self, req):
        """Requests with equal keys can run as one transform call (batched
        2-D inputs; a 1-D single map stays on its own)."""
        if req.data.dim() != 2:
            return ("alone", id(req))
        return (req.direction, req.nside, req.lmax, req.data.dtype)

    def need_group(self, reqs):
        """(transient, resident) bytes of one call on the requests' channels:
        outputs, workspace, the concatenated input when there are several,
        and the tables of an (nside, lmax) not yet resident."""
        from . import _lib
        r0 = reqs[0]
        code = self._code(r0)
        L = _lib.lib()
        B = sum(r.batch for r in reqs)
        ws = L.shtx_workspace_bytes(r0.nside, r0.lmax, B, code)
        cat = sum(r.data.numel() * r.data.element_size() for r in reqs) if len(reqs) > 1 else 0
        with self._tables_lock:
            known = (r0.nside, r0.lmax) in self._tables
        tab = 0 if known else L.shtx_tables_bytes(r0.nside, r0.lmax)
        return sum(self._out_bytes(r) for r in reqs) + ws + cat, tab

    def launch(self, req, slot):
        return self.launch_group([req], slot)

    def launch_group(self, reqs, slot):
        """One transform call on the channels of `reqs` (same group key),
        each request's result a slice of the output."""
        torch, ops = self.torch, self.ops
        req = reqs[0]
        key = (req.nside, req.lmax)
        with self._tables_lock:
            ev_tab = self._tables.get(key)
            if ev_tab is None:
                # built on the table stream; requests wait for that event on
                # their own streams (no device-wide synchronisation)
                with torch.cuda.stream(self.table_stream):
                    ops.get_tables(req.nside, req.lmax, self.device)
                    ev_tab = torch.cuda.Event()
                    ev_tab.record(self.table_stream)
                self._tables[key] = ev_tab
        st = self.streams[slot]
        st.wait_event(ev_tab)
        st.wait_stream(torch.cuda.current_stream(self.device))  # inputs written before submit
        with torch.cuda.stream(st):
            x = req.data if len(reqs) == 1 else torch.cat([r.data for r in reqs], dim=0)
            if req.direction == "map2alm":
                out = ops.map2alm_raw(x, req.lmax)
            else:
                out = ops.alm2map_raw(x, req.nside, req.lmax)
            ev = torch.cuda.Event()
            ev.record(st)
        if len(reqs) == 1:
            return (ev, out, None)
        bounds = []
        b = 0
        for r in reqs:
            bounds.append((b, b + r.batch))
            b += r.batch
        return (ev, out, bounds)

    def done(self, handle):
        return handle[0].query()

    def finish(self, handle):
        handle[0].synchronize()
        ev, out, bounds = handle
        if bounds is None:
            return out
        return [out[a:b] for a, b in bounds]


class Server:
    """GPU serving loop: `submit(Request) -> Future` of the output tensor."""

    def __init__(self, device="cuda:0", budget_bytes=48 << 30, slots=4, max_merge_channels=64):
        self.executor = GpuExecutor(device, slots)
        self.scheduler = Scheduler(self.executor, budget_bytes, slots, max_merge_channels=max_merge_channels)

    def submit(self, req):
        return self.scheduler.submit(req)

    def stats(self, t0=None, t1=None):
        return self.scheduler.stats(t0, t1)

    def drain(self):
        self.scheduler.drain()

    def close(self):
        self.scheduler.close()
