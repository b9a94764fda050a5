"""Serving loop: continuous batching of compressed time frames.

Requests (one frame each, device-resident or host arrays) arrive at any time.
The scheduler keeps up to `slots` batches in flight, each on its own stream
(default priority).  Whenever a slot is free it admits the oldest waiting
requests whose buffers fit the HBM budget -- up to `max_batch` of them -- and
decodes them together with one multi-frame plan; frames admitted while other
batches are still running overlap with them on the device.  A request's
latency runs from its arrival to the completion event of its batch.

All decoding is done by libtmd (through paper_2411_02206_amd.Plan); this
module only schedules.  Plans are cached per slot by their tuple of frame
shapes: calls on one plan are serialised by the library, so slots never share
one.
"""
import collections
import threading
import time

from . import Plan, alloc_out, frame_shape, to_device

# bytes of the device buffers of one frame: inputs, outputs and workspace (the
# workspace is taken from the plan once known; this estimate is used for
# admission before the plan exists)
IN_BYTES_TRACK = 15
IN_BYTES_CLUSTER = 10
OUT_BYTES_CLUSTER = 10
WS_BYTES_ATTACHED = 16 + 4        # records + start
WS_BYTES_TRACK = 4 + 4 + 1 + 90   # start, order, key, histogram rows
FIXED_BYTES = 5472 * 16 + (1 << 20)


def frame_bytes(shape):
    nT, nA, nU = shape
    return (nT * IN_BYTES_TRACK + (nA + nU) * (IN_BYTES_CLUSTER + OUT_BYTES_CLUSTER)
            + nA * WS_BYTES_ATTACHED + nT * WS_BYTES_TRACK + FIXED_BYTES)


class Request:
    __slots__ = ("frame", "shape", "arrival", "admitted", "done_time", "out", "flags", "event", "nbytes",
                 "on_device")

    def __init__(self, frame, arrival):
        self.frame = frame
        self.shape = frame_shape(frame)
        self.arrival = arrival
        self.admitted = None
        self.done_time = None
        self.out = None
        self.flags = None
        self.event = None
        self.nbytes = frame_bytes(self.shape)
        self.on_device = bool(getattr(frame["trk_ncls"], "is_cuda", False))

    @property
    def latency(self):
        return None if self.done_time is None else self.done_time - self.arrival


class _Batch:
    def __init__(self, reqs, plan, stream, event, ws, keep, slot):
        self.slot = slot
        self.reqs = reqs
        self.plan = plan
        self.stream = stream
        self.event = event
        self.ws = ws
        self.keep = keep


class Server:
    """Continuous-batching decoder.  submit() may be called from any thread;
    the scheduling runs in step()/run_until() on the calling thread (or
    start() for a background thread)."""

    def __init__(self, bz=0.5, hbm_budget=200e9, slots=4, max_batch=8, graph=False, device="cuda",
                 plan_cache=64, executor=None):
        self.bz = bz
        self.budget = float(hbm_budget)
        self.max_batch = max_batch
        self.peak_in_use = 0.0
        self.graph = graph
        self.device = device
        self.in_use = 0.0
        self.waiting = collections.deque()
        self.done = []
        self.lock = threading.Lock()
        self._plans = collections.OrderedDict()
        self._plan_cache = plan_cache
        self._busy = []
        self._executor = executor  # test hook: decodes a list of requests without a GPU
        if executor is None:
            import torch
            self._torch = torch
            self._streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        else:
            self._torch = None
            self._streams = [None] * slots
        self._free = list(range(slots))
        self._thread = None
        self._stop = False

    # -- client side ---------------------------------------------------------
    def submit(self, frame, arrival=None):
        r = Request(frame, time.perf_counter() if arrival is None else arrival)
        if r.nbytes > self.budget:
            raise ValueError(f"frame needs {r.nbytes:.3g} B, more than the HBM budget {self.budget:.3g} B")
        with self.lock:
            self.waiting.append(r)
        return r

    # -- scheduler -----------------------------------------------------------
    def _plan(self, slot, shapes):
        key = (slot, tuple(shapes))
        p = self._plans.get(key)
        if p is not None:
            self._plans.move_to_end(key)
            return p
        from . import PLAN_GRAPH
        p = Plan(shapes, bz=self.bz, flags=PLAN_GRAPH if self.graph else 0)
        self._plans[key] = p
        while len(self._plans) > self._plan_cache:
            _, old = self._plans.popitem(last=False)
            old.free()
        return p

    def _retire(self):
        still = []
        for b in self._busy:
            finished = b.event is None or b.event.query()
            if finished:
                now = time.perf_counter()
                for i, r in enumerate(b.reqs):
                    r.done_time = now
                    if b.plan is not None:
                        r.flags = b.plan.status(i)
                    self.in_use -= r.nbytes
                    self.done.append(r)
                self._free.append(b.slot)
            else:
                still.append(b)
        self._busy = still

    def _admit(self):
        if not self._free:
            return False
        batch = []
        with self.lock:
            while self.waiting and len(batch) < self.max_batch:
                r = self.waiting[0]
                if self.in_use + r.nbytes > self.budget:
                    break
                self.waiting.popleft()
                self.in_use += r.nbytes
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                batch.append(r)
        if not batch:
            return False
        slot = self._free.pop()
        now = time.perf_counter()
        for r in batch:
            r.admitted = now
        if self._executor is not None:
            self._executor(batch)
            self._busy.append(_Batch(batch, None, None, None, None, None, slot))
            return True
        torch = self._torch
        stream = self._streams[slot]
        shapes = [r.shape for r in batch]
        plan = self._plan(slot, shapes)
        with torch.cuda.stream(stream):
            ins = [r.frame if r.on_device else to_device(r.frame, self.device) for r in batch]
            outs = [alloc_out(r.shape, self.device) for r in batch]
            ws = plan.alloc_workspace(self.device)
            plan.decode(ins, outs, ws, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r, o in zip(batch, outs):
            r.out = o
        self._busy.append(_Batch(batch, plan, stream, ev, ws, ins, slot))
        return True

    def step(self):
        """One scheduling round: retire finished batches, admit new ones.
        Returns True if anything is waiting or in flight."""
        self._retire()
        while self._admit():
            pass
        with self.lock:
            return bool(self.waiting) or bool(self._busy)

    def run_until(self, n_done, timeout=600.0):
        t_end = time.perf_counter() + timeout
        while len(self.done) < n_done:
            self.step()
            if time.perf_counter() > t_end:
                raise TimeoutError(f"served {len(self.done)} of {n_done} requests")
            time.sleep(0)
        return self.done

    def start(self):
        def loop():
            while not self._stop:
                if not self.step():
                    time.sleep(50e-6)
        self._stop = False
        self._thread = threading.Thread(target=loop, daemon=True)
        self._thread.start()

    def stop(self):
        self._stop = True
        if self._thread is not None:
            self._thread.join()
            self._thread = None

    def close(self):
        self.stop()
        for p in self._plans.values():
            p.free()
        self._plans.clear()


def percentile(values, q):
    v = sorted(values)
    if not v:
        return None
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)
