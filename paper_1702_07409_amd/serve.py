"""Request loop with continuous batching over the batched plans.

Requests (encode, decode, repair, update) arrive over time.  Every pass of
the loop (a "tick"):

  1. observes which launched ticks have completed (a HIP event per tick),
     finishes their requests and releases their memory and stripe locks;
  2. admits pending requests in arrival order while their device footprint
     fits the budget (a request that does not fit stops admission, so large
     requests are not starved), skipping requests whose graph is still being
     built or whose stripe is held by an earlier request;
  3. packs the admitted requests into one plan in device memory taken from
     torch (fs_plan_create_in: descriptors copied from pinned host memory,
     no hipMalloc, no stream sync) and launches it on the next of a few
     rotating streams, so ticks overlap on the device.

Graphs are kept on the device in a cache keyed by their parameters (the
paper regenerates an object's graph from its seed and parameters, so objects
of equal k and n share one).  A missing graph is built when its request
arrives, on a thread pool so that the loop goes on: by kernels on the
device (fs_graph_build with FS_GRAPH_ON_DEVICE, each worker on a stream of
its own; the call returns with the graph complete), or, with device builds
off, on the host, the device copy then being made on the stream of the tick
that first uses it, other streams waiting for that copy.

The loop and the build threads share the interpreter lock: the loop polls
without blocking, and a thread that waits for the lock gets it only when
the holder has run for the interpreter's switch interval (5 ms by default).
run() therefore shortens the switch interval (switch_interval, 50 us) for
its duration, so that a build starts and finishes without waiting on the
loop.  It also turns off the interpreter's cyclic garbage collector for its
duration (pause_gc): a collection of the young generations stops every
thread for 0.5-1 ms, about the device time of a large request, and the
loop's objects are freed by reference counting anyway.  Before it starts,
run() takes the in-flight budget from torch's caching allocator once and
gives it back (reserve), so that the outputs and plans of the requests are
carved from memory the allocator already holds instead of new device
allocations in the middle of the run (a first run without it showed stalls
of several milliseconds).

Resident stripes (inputs x and coded blocks c kept on the device) are the
targets of decode, repair (from the resident inputs) and update.  Requests on
one stripe run one at a time in arrival order.

Everything on the device runs in libfs.so; this module only schedules.
"""

import collections
import gc
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import torch

from . import _lib as fs

ENCODE, DECODE, REPAIR, UPDATE = "encode", "decode", "repair", "update"


def _empty(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class GraphEntry:
    """A graph in the cache: host build (future), device copy, readiness."""

    __slots__ = ("key", "future", "graph", "mem", "event", "stream", "refs", "bytes", "last")

    def __init__(self, key, future):
        self.key = key
        self.future = future
        self.graph = None
        self.mem = None          # device tensor holding the graph image
        self.event = None        # completes when the device copy has landed
        self.stream = None       # stream the copy was made on
        self.refs = 0            # pending and in-flight requests and resident stripes using it
        self.bytes = 0
        self.last = 0.0

    def ready(self):
        return self.graph is not None or self.future.done()


class GraphCache:
    """Device graphs keyed by their parameters, with LRU eviction of unused
    entries beyond `capacity` bytes."""

    def __init__(self, device, workers=8, capacity=4 << 30, device_builds=True):
        self.device = device
        self.device_builds = device_builds
        self.local = threading.local()
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.capacity = capacity
        self.entries = collections.OrderedDict()
        self.device_bytes = 0
        self.builds = 0
        self.hits = 0

    @staticmethod
    def key_of(params):
        return tuple(sorted(params.items()))

    def prefetch(self, params):
        key = self.key_of(params)
        e = self.entries.get(key)
        if e is None:
            p = dict(params)
            p["finite_w"] = tuple(p.get("finite_w", ()))
            if self.device_builds:
                e = GraphEntry(key, self.pool.submit(self._build_on_device, p))
            else:
                e = GraphEntry(key, self.pool.submit(fs.fs_graph_build, host_only=True, **p))
            self.entries[key] = e
            self.builds += 1
        else:
            self.hits += 1
            self.entries.move_to_end(key)
        return e

    def _build_on_device(self, p):
        # a worker thread: its own stream (the build waits on it)
        s = getattr(self.local, "stream", None)
        if s is None:
            s = self.local.stream = torch.cuda.Stream(device=self.device)
        return fs.fs_graph_build(on_device=True, stream=s, **p)

    def on_device(self, e, stream, keep):
        """Make sure e has a device copy usable on `stream`; pinned staging
        buffers that must outlive the copy are appended to `keep`."""
        if e.graph is None:
            e.graph = e.future.result()
        if e.graph.built_on_device:
            if not e.bytes:   # complete on the device when its build returned
                e.bytes = e.graph.device_bytes()
                self.device_bytes += e.bytes
        elif e.mem is None:
            nbytes = e.graph.image_size()
            e.mem = _empty(nbytes, self.device)
            stage = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
            e.graph.upload(e.mem, stage=stage, stream=stream)
            keep.append(stage)
            e.event = torch.cuda.Event()
            e.event.record(stream)
            e.stream = stream
            e.bytes = nbytes
            self.device_bytes += nbytes
        elif e.event is not None and e.stream is not stream:
            if e.event.query():
                e.event = None
            else:
                stream.wait_event(e.event)
        e.last = time.perf_counter()

    def evict(self):
        while self.device_bytes > self.capacity:
            victim = None
            for key, e in self.entries.items():
                if e.refs == 0 and e.bytes:
                    victim = key
                    break
            if victim is None:
                return
            e = self.entries.pop(victim)
            self.device_bytes -= e.bytes
            e.graph.free()
            e.mem = None

    def close(self):
        self.pool.shutdown(wait=True)


class Stripe:
    """A resident stripe: inputs x[k][t] and coded blocks c[n][t] on the device."""

    def __init__(self, sid, entry, x, c, t):
        self.sid = sid
        self.entry = entry
        self.x, self.c, self.t = x, c, t


class Request:
    """One request.  Encode: params (graph parameters), t, x (device input
    blocks).  Decode: stripe, erased (device uint8[n]), maxit.  Repair:
    stripe, ids (device uint32 lost coded rows).  Update: stripe, ids (device
    uint32 input ids), new_blocks (device [n_ids][t])."""

    def __init__(self, kind, arrival=0.0, params=None, t=0, x=None, stripe=None, erased=None, maxit=0,
                 ids=None, new_blocks=None, rid=None):
        self.kind = kind
        self.arrival = arrival
        self.params, self.t, self.x = params, t, x
        self.stripe, self.erased, self.maxit = stripe, erased, maxit
        self.ids, self.new_blocks = ids, new_blocks
        self.rid = rid
        # results
        self.c = None          # encode: coded blocks
        self.out = None        # decode: decoded inputs
        self.recovered = None  # decode: uint8[k]
        self.status = None     # decode / repair / update: int32[3] (device)
        self.repaired = None   # repair: uint8[m]
        # bookkeeping
        self.entry = None
        self.footprint = 0
        self.user_bytes = 0
        self.t_submit = None
        self.t_launch = None
        self.t_done = None
        self.tick = None


class Tick:
    __slots__ = ("requests", "plan", "keep", "stream", "start", "end", "footprint", "t_launch")


class Scheduler:
    """Admission of pending requests (host logic only, no device calls).

    Requests are admitted in arrival order while their footprint fits the
    budget; the first one that does not fit stops admission (unless nothing
    is in flight and the tick is empty: a request larger than the whole
    budget then runs alone), so large requests are not starved.  A request
    is skipped (it stays pending, later ones may pass it) while its graph is
    not built yet, or while its stripe is held by an earlier request: each
    stripe serves its requests one at a time in arrival order.

    footprint(r): device bytes request r holds while in flight.
    """

    def __init__(self, budget, max_items, footprint):
        self.budget = budget
        self.max_items = max_items
        self.footprint = footprint
        self.pending = collections.deque()
        self.used = 0
        self.busy = set()                  # stripes held by an in-flight request
        self.queues = {}                   # stripe -> its pending requests, in arrival order

    def submit(self, r):
        if r.stripe is not None:
            self.queues.setdefault(r.stripe, collections.deque()).append(r)
        self.pending.append(r)

    def eligible(self, r):
        if not r.entry.ready():
            return False
        if r.stripe is None:
            return True
        return r.stripe not in self.busy and self.queues[r.stripe][0] is r

    def admit(self, inflight):
        """Requests for the next tick (their footprint is charged)."""
        batch, rest = [], collections.deque()
        blocked = False
        while self.pending:
            r = self.pending.popleft()
            if blocked or len(batch) >= self.max_items or not self.eligible(r):
                rest.append(r)
                continue
            fp = self.footprint(r)
            if self.used + fp > self.budget and (inflight or batch):
                blocked = True   # keep arrival order for memory
                rest.append(r)
                continue
            r.footprint = fp
            self.used += fp
            if r.stripe is not None:
                self.busy.add(r.stripe)
            batch.append(r)
        self.pending = rest
        return batch

    def release(self, r):
        """Request r has completed: free its footprint and its stripe."""
        self.used -= r.footprint
        if r.stripe is not None:
            self.busy.discard(r.stripe)
            self.queues[r.stripe].popleft()


class Server:
    """Continuous-batching request loop on one GPU.

    budget: device bytes that in-flight requests may hold (outputs and the
    plans with their workspaces; the plan of a tick is counted once the tick
    is formed, so one tick may exceed the budget by its plan); streams: rotating launch streams; max_inflight:
    ticks on the device at once; max_items: requests per tick.
    """

    def __init__(self, budget=32 << 30, streams=3, max_inflight=4, max_items=64, workers=8,
                 graph_cache_bytes=4 << 30, keep_outputs=False, device="cuda", device_graph_builds=True,
                 switch_interval=50e-6, pause_gc=True, reserve=True):
        self.device = torch.device(device)
        self.switch_interval = switch_interval
        self.pause_gc = pause_gc
        self.reserve = reserve
        self.budget = budget
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.next_stream = 0
        self.max_inflight = max_inflight
        self.max_items = max_items
        self.keep_outputs = keep_outputs
        self.cache = GraphCache(self.device, workers, graph_cache_bytes, device_graph_builds)
        self.stripes = {}
        self.sched = Scheduler(budget, max_items, self._footprint)
        self.inflight = collections.deque()
        self.done = []
        self.ticks = 0
        self.tick_items = []
        self.busy_events = []   # (start, end) events of each tick
        self.ref = None
        self.peak_inflight = 0

    # ---------------------------------------------------------------- setup

    def add_stripe(self, sid, params, x, c, t):
        """Register a resident stripe whose coded blocks c are already the
        encoding of x (as made by encode_now)."""
        e = self.cache.prefetch(params)
        s = torch.cuda.current_stream(self.device)
        keep = []
        self.cache.on_device(e, s, keep)
        e.refs += 1   # resident stripes pin their graph
        st = Stripe(sid, e, x, c, t)
        self.stripes[sid] = st
        return st

    def encode_now(self, params, x, t):
        """Encode x with the cached graph of `params` on the current stream
        (for filling the resident pool) and return c."""
        e = self.cache.prefetch(params)
        s = torch.cuda.current_stream(self.device)
        self.cache.on_device(e, s, [])
        g = e.graph
        c = torch.empty((g.n, t), dtype=torch.uint8, device=self.device)
        fs.fs_encode(g, x, c, t, stream=s)
        return c

    # ---------------------------------------------------------------- requests

    def submit(self, r):
        """A request arrives (device inputs already in place)."""
        r.t_submit = time.perf_counter()
        if r.kind == ENCODE:
            r.entry = self.cache.prefetch(r.params)
            r.stripe = None
        else:
            r.entry = self.stripes[r.stripe].entry
        r.entry.refs += 1
        self.sched.submit(r)

    def _footprint(self, r):
        """Device bytes of the request's outputs (its workspace is part of the
        tick's plan memory, counted when the tick is launched)."""
        if r.entry.graph is None:
            r.entry.graph = r.entry.future.result()
        g = r.entry.graph
        if r.kind == ENCODE:
            return g.n * r.t + 1024
        if r.kind == DECODE:
            return g.k * r.t + g.k + 1024
        return int(r.ids.numel()) + 1024

    def _items(self, batch, stream, keep):
        items = []
        dev = self.device
        for r in batch:
            self.cache.on_device(r.entry, stream, keep)
            g = r.entry.graph
            if r.kind == ENCODE:
                r.c = torch.empty((g.n, r.t), dtype=torch.uint8, device=dev)
                items.append(fs.work(ENCODE, g, r.t, x=r.x, c=r.c))
                r.user_bytes = g.k * r.t
                continue
            st = self.stripes[r.stripe]
            r.status = torch.empty(4, dtype=torch.int32, device=dev)
            if r.kind == DECODE:
                r.out = torch.empty((g.k, r.t), dtype=torch.uint8, device=dev)
                r.recovered = torch.empty(g.k, dtype=torch.uint8, device=dev)
                items.append(fs.work(DECODE, g, r.t, x=r.out, c=st.c, erased=r.erased, maxit=r.maxit,
                                     recovered=r.recovered, status=r.status))
            elif r.kind == REPAIR:
                m = int(r.ids.numel())
                r.repaired = torch.empty(m, dtype=torch.uint8, device=dev)
                items.append(fs.work(REPAIR, g, r.t, x=st.x, c=st.c, ids=r.ids, n_ids=m,
                                     repaired=r.repaired, status=r.status))
                r.user_bytes = m * r.t
            else:
                m = int(r.ids.numel())
                items.append(fs.work(UPDATE, g, r.t, x=st.x, c=st.c, ids=r.ids, n_ids=m,
                                     new_blocks=r.new_blocks, status=r.status))
                r.user_bytes = m * r.t
        return items

    def _launch(self, batch):
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        tk = Tick()
        tk.keep = []
        tk.requests = batch
        tk.stream = stream
        tk.start = torch.cuda.Event(enable_timing=True)
        tk.end = torch.cuda.Event(enable_timing=True)
        tk.start.record(stream)
        items = self._items(batch, stream, tk.keep)
        dev_bytes, stage_bytes = fs.plan_memory_size(items)
        mem = _empty(dev_bytes, self.device)
        stage = torch.empty(max(stage_bytes, 1), dtype=torch.uint8, pin_memory=True)
        tk.plan = fs.Plan(items, memory=mem, stage=stage, stream=stream)
        tk.plan.launch(stream=stream)
        tk.end.record(stream)
        tk.keep += [mem, stage, items]
        tk.footprint = dev_bytes
        self.sched.used += dev_bytes
        tk.t_launch = time.perf_counter()
        for r in batch:
            r.t_launch = tk.t_launch
            r.tick = self.ticks
        self.inflight.append(tk)
        self.peak_inflight = max(self.peak_inflight, len(self.inflight))
        self.busy_events.append((tk.start, tk.end))
        self.ticks += 1
        self.tick_items.append(len(batch))

    def _complete(self, tk, now):
        tk.plan.free()
        self.sched.used -= tk.footprint
        for r in tk.requests:
            r.t_done = now
            self.sched.release(r)
            r.entry.refs -= 1
            if not self.keep_outputs:
                r.c = r.out = None
            self.done.append(r)
        tk.keep = None

    def poll(self):
        """Finish every launched tick whose work has completed (in order per stream)."""
        now = time.perf_counter()
        still = collections.deque()
        finished = False
        for tk in self.inflight:
            if tk.end.query():
                self._complete(tk, now)
                finished = True
            else:
                still.append(tk)
        self.inflight = still
        if finished:
            self.cache.evict()
        return finished

    def step(self):
        """One pass of the loop; returns True when it launched a tick."""
        self.poll()
        if not self.sched.pending or len(self.inflight) >= self.max_inflight:
            return False
        batch = self.sched.admit(len(self.inflight))
        if not batch:
            return False
        self._launch(batch)
        return True

    def drain(self):
        while self.sched.pending or self.inflight:
            if not self.step():
                time.sleep(0)

    # ---------------------------------------------------------------- driver

    def run(self, requests, time_scale=1.0):
        """Serve `requests` (sorted by .arrival, seconds from the start);
        each is submitted once the wall clock passes its arrival time scaled
        by time_scale.  Returns the statistics of the run.  The interpreter's
        thread switch interval is switch_interval while it runs (None: left
        as it is), and the cyclic garbage collector is off if pause_gc.  With
        reserve, the budget is first taken from torch's caching allocator and
        given back."""
        if self.reserve:
            self._reserve()
        prev = sys.getswitchinterval()
        if self.switch_interval:
            sys.setswitchinterval(self.switch_interval)
        gc_was = gc.isenabled()
        if self.pause_gc:
            gc.disable()
        try:
            return self._run(requests, time_scale)
        finally:
            sys.setswitchinterval(prev)
            if gc_was:
                gc.enable()

    def _reserve(self):
        """Hold the budget in torch's caching allocator (best effort: skipped
        when the device cannot spare it)."""
        try:
            block = torch.empty(max(int(self.budget), 1), dtype=torch.uint8, device=self.device)
        except torch.OutOfMemoryError:
            return
        del block

    def _run(self, requests, time_scale):
        torch.cuda.synchronize(self.device)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.streams[0])
        self.done = []
        self.busy_events = []
        self.tick_items = []
        t0 = time.perf_counter()
        i, nreq = 0, len(requests)
        while i < nreq or self.sched.pending or self.inflight:
            now = time.perf_counter() - t0
            while i < nreq and requests[i].arrival * time_scale <= now:
                self.submit(requests[i])
                i += 1
            if not self.step():
                time.sleep(0)
        torch.cuda.synchronize(self.device)
        t_end = time.perf_counter()
        return self.stats(requests, t0, t_end, time_scale)

    def busy_ms(self):
        """Union of the device intervals of the ticks (ms), from their events."""
        iv = sorted((self.ref.elapsed_time(a), self.ref.elapsed_time(b)) for a, b in self.busy_events)
        total, cur_s, cur_e = 0.0, None, None
        for s, e in iv:
            if cur_e is None or s > cur_e:
                if cur_e is not None:
                    total += cur_e - cur_s
                cur_s, cur_e = s, e
            else:
                cur_e = max(cur_e, e)
        if cur_e is not None:
            total += cur_e - cur_s
        return total

    def stats(self, requests, t0, t_end, time_scale):
        lat = sorted((r.t_done - (t0 + r.arrival * time_scale)) * 1e3 for r in requests)
        q = lambda p: lat[min(len(lat) - 1, int(p * len(lat)))] if lat else 0.0
        for r in requests:
            if r.kind == DECODE and r.recovered is not None:
                r.user_bytes = int(r.recovered.sum().item()) * r.t
        user = sum(r.user_bytes for r in requests)
        wall = t_end - t0
        busy = self.busy_ms()
        by_kind = {}
        for kind in (ENCODE, DECODE, REPAIR, UPDATE):
            lk = sorted((r.t_done - (t0 + r.arrival * time_scale)) * 1e3 for r in requests if r.kind == kind)
            if lk:
                by_kind[kind] = {"count": len(lk), "p50_ms": round(lk[len(lk) // 2], 3),
                                 "p99_ms": round(lk[min(len(lk) - 1, int(0.99 * len(lk)))], 3)}
        return {
            "requests": len(requests),
            "wall_s": round(wall, 4),
            "req_per_s": round(len(requests) / wall, 1),
            "user_GB": round(user / 1e9, 3),
            "user_GBps_wall": round(user / wall / 1e9, 2),
            "busy_ms": round(busy, 2),
            "user_GBps_busy": round(user / (busy * 1e-3) / 1e9, 2) if busy > 0 else None,
            "p50_ms": round(q(0.50), 3),
            "p99_ms": round(q(0.99), 3),
            "max_ms": round(lat[-1], 3) if lat else 0.0,
            "ticks": len(self.tick_items),
            "mean_items_per_tick": round(sum(self.tick_items) / max(1, len(self.tick_items)), 2),
            "graph_builds": self.cache.builds,
            "graph_hits": self.cache.hits,
            "by_kind": by_kind,
        }

    def close(self):
        self.cache.close()
