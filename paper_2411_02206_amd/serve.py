"""Serving loop: continuous batching of compressed time frames.

Requests (one frame each, device-resident or host arrays) arrive at any time.
The scheduler keeps up to `slots` batches in flight, each on its own stream
(default priority).  Whenever a slot is free it admits the oldest waiting
requests whose buffers fit the HBM budget -- up to `max_batch` of them -- and
decodes them together with one launch sequence; batches admitted while
others are still running overlap with them on the device.  A request's
latency runs from its arrival to the moment its batch's completion event was
reached on the device (read from the event's timestamp, not from when the
scheduler next looked).

Each slot owns plans whose frame shapes are capacities (tmd_decode_shapes):
one per batch size 1, 2, 4, ... up to max_batch, each with that many entries
of the server's per-frame capacity.  A batch of b frames uses the smallest
plan with at least b entries and leaves its remaining entries idle, so few
idle entries are launched, and the plans, the slot's one workspace (sized for
its largest plan) and (with graph=True) their captured HIP graphs are made
once and reused.  The capacity starts at the first frame's shape times 1.25
(or is given) and grows by the same factor when a larger frame arrives; a
slot rebuilds its plans when it is next used.  The HBM budget covers the
requests' buffers and the slots' workspaces: a slot whose plans must be
rebuilt admits a batch only if the new workspace fits as well.  `warm()`
builds every slot's plans and graphs ahead of the traffic.  All decoding is
done by libtmd; this module schedules.
"""
import collections
import threading
import time

from . import IN_FIELDS, NBIN, PLAN_GRAPH, Plan, alloc_out, frame_shape, to_device

# bytes of the device buffers of one request: inputs (when copied in) and outputs
IN_BYTES_TRACK = 15
IN_BYTES_CLUSTER = 10
OUT_BYTES_CLUSTER = 10
FIXED_BYTES = (2 * NBIN + 1) * 4 + (1 << 12)
GROWTH = 1.25


def frame_bytes(shape, inputs=True):
    nT, nA, nU = shape
    b = (nA + nU) * OUT_BYTES_CLUSTER + FIXED_BYTES
    if inputs:
        b += nT * IN_BYTES_TRACK + (nA + nU) * IN_BYTES_CLUSTER
    return b


def _grow(cap, shape):
    return tuple(max(c, int(s * GROWTH) + 1) if s > c else c for c, s in zip(cap, shape))


def batch_sizes(max_batch):
    """Entries of a slot's plans: 1, 2, 4, ... and max_batch."""
    sizes, b = [], 1
    while b < max_batch:
        sizes.append(b)
        b *= 2
    sizes.append(max_batch)
    return sizes


class Request:
    __slots__ = ("frame", "shape", "arrival", "admitted", "done_time", "out", "flags", "nbytes", "on_device")

    def __init__(self, frame, arrival):
        self.frame = frame
        self.shape = frame_shape(frame)
        self.arrival = arrival
        self.admitted = None
        self.done_time = None
        self.out = None
        self.flags = None
        self.on_device = bool(getattr(frame["trk_ncls"], "is_cuda", False))
        self.nbytes = frame_bytes(self.shape, inputs=not self.on_device)

    @property
    def latency(self):
        return None if self.done_time is None else self.done_time - self.arrival


class _Slot:
    """A stream with its capacity plans, workspace and idle-entry buffers."""

    def __init__(self, stream):
        self.stream = stream
        self.plans = {}    # entries -> Plan
        self.ws = None
        self.ws_bytes = 0  # reserved in the server's budget
        self.cap = None
        self.idle_in = None
        self.idle_out = None
        self.reqs = None   # the batch in flight, if any
        self.plan = None   # its plan
        self.event = None
        self.keep = None   # its input buffers


class Server:
    """Continuous-batching decoder.  submit() may be called from any thread;
    the scheduling runs in step()/run_until() on the calling thread (or
    start() for a background thread).  capacity: per-frame (n_tracks,
    n_attached, n_unattached) of the slot plans, or None to size them from
    the frames that arrive.  schedule: (tracks per wave, persistent waves per
    SIMD) for the plans' attached decode (see Plan.set_schedule)."""

    def __init__(self, bz=0.5, hbm_budget=200e9, slots=4, max_batch=8, graph=False, device="cuda",
                 capacity=None, executor=None, schedule=None):
        self.bz = bz
        self.budget = float(hbm_budget)
        self.max_batch = max_batch
        self.sizes = batch_sizes(max_batch)
        self.graph = graph
        self.device = device
        self.schedule = schedule
        self.capacity = tuple(capacity) if capacity is not None else None
        self.peak_in_use = 0.0
        self.in_use = 0.0
        self.waiting = collections.deque()
        self.done = []
        self.lock = threading.Lock()
        self._executor = executor  # test hook: decodes a list of requests without a GPU
        if executor is None:
            import torch
            self._torch = torch
            self._slots = [_Slot(torch.cuda.Stream(device=device)) for _ in range(slots)]
            # device clock reference: completion times are this host time
            # plus the device time elapsed since the reference event
            self._ref = torch.cuda.Event(enable_timing=True)
            self._ref.record(self._slots[0].stream)
            self._ref.synchronize()
            self._ref_host = time.perf_counter()
        else:
            self._torch = None
            self._slots = [_Slot(None) for _ in range(slots)]
        self._free = list(range(slots))
        self._busy = []  # slot indices with a batch in flight
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
    def _build(self, S, cap):
        """Plans of slot S for capacity `cap`; returns their workspace bytes
        (the workspace itself is allocated by _commit)."""
        for p in S.plans.values():
            p.free()
        S.plans = {}
        flags = PLAN_GRAPH if self.graph else 0
        for b in self.sizes:
            p = Plan([cap] * b, bz=self.bz, flags=flags)
            if self.schedule is not None:
                p.set_schedule(*self.schedule)
            S.plans[b] = p
        return max(p.workspace_bytes for p in S.plans.values())

    def _commit(self, S, cap, ws_bytes):
        torch = self._torch
        if S.ws is not None:
            self.in_use -= S.ws_bytes
            S.ws = None
        S.cap = cap
        S.ws_bytes = ws_bytes
        with torch.cuda.stream(S.stream):
            S.ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=self.device)
            if S.idle_in is None:
                S.idle_in = {k: None for k in IN_FIELDS}
                S.idle_in["un_count"] = torch.zeros(NBIN, dtype=torch.int32, device=self.device)
                o = alloc_out((0, 0, 0), self.device)
                S.idle_out = {k: (o[k] if k in ("row_offset", "row_nattached") else None) for k in o}
                S.idle_out["capacity"] = 0
        self.in_use += ws_bytes
        self.peak_in_use = max(self.peak_in_use, self.in_use)

    def warm(self, capacity=None):
        """Build every slot's plans for `capacity` (default: the server's) and
        replay each plan once on idle entries, so that plan creation and graph
        capture happen before the traffic."""
        if capacity is not None:
            self.capacity = tuple(capacity)
        if self._executor is not None or self.capacity is None:
            return
        for S in self._slots:
            if S.cap != self.capacity:
                ws = self._build(S, self.capacity)
                self._commit(S, self.capacity, ws)
            for b, p in S.plans.items():
                p.decode([S.idle_in] * b, [S.idle_out] * b, S.ws, S.stream, shapes=[(0, 0, 0)] * b)
        self._torch.cuda.synchronize()

    def _done_time(self, S):
        if self._executor is not None or S.event is None:
            return time.perf_counter()
        return self._ref_host + self._ref.elapsed_time(S.event) * 1e-3

    def _retire(self):
        still = []
        for si in self._busy:
            S = self._slots[si]
            if S.event is None or S.event.query():
                t = self._done_time(S)
                for i, r in enumerate(S.reqs):
                    r.done_time = t
                    if S.plan is not None and self._executor is None:
                        r.flags = S.plan.status(i)
                    self.in_use -= r.nbytes
                    self.done.append(r)
                S.reqs, S.event, S.keep, S.plan = None, None, None, None
                self._free.append(si)
            else:
                still.append(si)
        self._busy = still

    def _admit(self):
        if not self._free:
            return False
        si = self._free[-1]
        S = self._slots[si]
        batch = []
        cap = self.capacity
        rebuild_ws = None  # workspace bytes of the slot's plans for `cap`, if they must be rebuilt
        with self.lock:
            while self.waiting and len(batch) < self.max_batch:
                r = self.waiting[0]
                new_cap = _grow((0, 0, 0), r.shape) if cap is None else (
                    _grow(cap, r.shape) if any(s > c for s, c in zip(r.shape, cap)) else cap)
                extra = 0.0
                if self._executor is None and new_cap != S.cap:
                    if new_cap != cap or rebuild_ws is None:
                        rebuild_ws = self._build(S, new_cap)
                    extra = rebuild_ws - S.ws_bytes
                if self.in_use + r.nbytes + extra > self.budget:
                    break
                self.waiting.popleft()
                self.in_use += r.nbytes
                self.peak_in_use = max(self.peak_in_use, self.in_use + extra)
                batch.append(r)
                cap = new_cap
        if not batch:
            if S.plans and S.cap is not None and self._executor is None and rebuild_ws is not None:
                self._build(S, S.cap)  # the trial plans did not fit: back to the slot's own
            return False
        self.capacity = cap
        self._free.pop()
        now = time.perf_counter()
        for r in batch:
            r.admitted = now
        S.reqs = batch
        self._busy.append(si)
        if self._executor is not None:
            self._executor(batch)
            return True
        if S.cap != cap:
            if rebuild_ws is None:
                rebuild_ws = self._build(S, cap)
            self._commit(S, cap, rebuild_ws)
        torch = self._torch
        entries = next(b for b in self.sizes if b >= len(batch))
        S.plan = S.plans[entries]
        idle = entries - len(batch)
        with torch.cuda.stream(S.stream):
            ins = [r.frame if r.on_device else to_device(r.frame, self.device) for r in batch]
            outs = [alloc_out(r.shape, self.device) for r in batch]
            S.plan.decode(ins + [S.idle_in] * idle, outs + [S.idle_out] * idle, S.ws, S.stream,
                          shapes=[r.shape for r in batch] + [(0, 0, 0)] * idle)
            S.event = torch.cuda.Event(enable_timing=True)
            S.event.record(S.stream)
        for r, o in zip(batch, outs):
            r.out = o
        S.keep = ins
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
        if self._torch is not None:
            self._torch.cuda.synchronize()
        for S in self._slots:
            for p in S.plans.values():
                p.free()
            S.plans = {}
            S.plan = None
            S.ws = None


def percentile(values, q):
    v = sorted(values)
    if not v:
        return None
    k = (len(v) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (k - lo)
