"""Continuous batching of many tracking streams on one GPU.

Streams arrive over time.  Each has its own video whose frames arrive at a
fixed rate, its own particle count, precision mode and motion model, and runs
the per-frame SIR step of the library (paper Sec. 2 and Sec. 4) on every frame.
The server:

  * admits a stream when a filter slot whose workspace share fits it is free
    (slots are pre-sized from a device-memory budget, so admission is the HBM
    budget check); otherwise the stream waits in a FIFO queue (first fit);
  * rejects at submission a stream whose parameters the library refuses;
  * at every tick steps, with one batched launch per slot pool, every admitted
    stream that has a frame waiting (one frame per stream per tick, in order;
    a heap of the streams' next frame arrival times finds them without
    scanning the idle ones);
  * measures per-frame latency: frame arrival to estimate ready;
  * evicts a stream whose frames stop arriving for longer than a timeout, and
    a stream whose step failed, reclaiming the slot either way.

The scheduler is independent of the device: a backend provides slots, the
batched step and estimates.  Two GPU backends keep one `pf_batch` per
precision:

  * `GpuByteBackend` admits by bytes: every admitted stream gets exactly its
    workspace (pf_member_bytes of its parameters) from a per-precision
    device arena of the HBM budget (first fit, freed ranges coalesce), and a
    batch member is rebound to that share (pf_batch_rebind); a stream waits
    only when no free range of the arena holds its bytes (or every member
    handle is taken);
  * `GpuPoolBackend` pre-sizes slots in power-of-two particle classes and
    re-initialises a free slot in place (pf_batch_reinit): simpler, but a
    burst of large streams waits while small slots sit idle.

A HIP error in a batched step poisons that pool's batch, so every stream
stepping in it fails; the scheduler then fails exactly those streams.
"""
from __future__ import annotations

import bisect
import heapq
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import (PF_F16, PF_F32, PF_F64, PF_BF16, Batch, PfError, make_params, pf_params,
               pf_member_bytes)

WS_ALIGN = 256  # workspace shares start on 256-byte boundaries


@dataclass
class StreamRequest:
    """One tracking stream.  Frame i (1 <= i < n_frames) arrives at
    arrival + i / fps; frame 0 is the known starting position (params.x0, y0).
    frame(i) returns the device frame (or host frame for a host backend), or
    None while the source stalls."""
    sid: int
    arrival: float
    params: pf_params
    n_frames: int
    fps: float
    frame: object  # callable i -> frame or None
    truth: object = None  # optional callable i -> (x, y)


@dataclass
class FrameSeq:
    """Frames at a fixed stride in device memory: frame i starts at
    base + i * stride, its rows `pitch` bytes apart.  A frame source like any
    other (calling it gives the (pointer, pitch) pair); over a backend with
    the array calls (step_arrays) the scheduler steps such streams from
    columns of numbers, with no per-stream Python work in a tick."""
    base: int
    stride: int
    pitch: int

    def __call__(self, i):
        return (self.base + i * self.stride, self.pitch)


@dataclass
class _Live:
    req: StreamRequest
    slot: object
    admitted: float
    next_frame: int = 1
    estimates: list = field(default_factory=list)
    row: int = -1  # row in the scheduler's column table (FrameSeq streams), or -1


class _Columns:
    """The FrameSeq streams being served, one row each: the numbers a tick
    needs, as arrays, and their estimates in one store (each stream a
    contiguous run of n_frames - 1 rows, compacted when the store is full)."""

    def __init__(self, cap: int = 1024):
        self.cap = 0
        self.rows_top = 0
        self.free = []
        self._grow(cap)
        self.est = np.zeros((4 * cap, 2))
        self.top = 0

    def _grow(self, cap):
        def ext(a, dtype):
            out = np.zeros(cap, dtype=dtype)
            if a is not None:
                out[:a.size] = a
            return out
        g = lambda name: getattr(self, name, None)  # noqa: E731
        self.used = ext(g("used"), bool)
        self.sid = ext(g("sid"), np.int64)
        self.code = ext(g("code"), np.int64)
        self.member = ext(g("member"), np.int64)
        self.nxt = ext(g("nxt"), np.int64)
        self.nfr = ext(g("nfr"), np.int64)
        self.arr = ext(g("arr"), np.float64)
        self.fps = ext(g("fps"), np.float64)
        self.due = ext(g("due"), np.float64)
        self.base = ext(g("base"), np.int64)
        self.stride = ext(g("stride"), np.int64)
        self.pitch = ext(g("pitch"), np.int64)
        self.npart = ext(g("npart"), np.int64)
        self.eoff = ext(g("eoff"), np.int64)
        self.cap = cap

    def _alloc_est(self, m):
        if self.top + m > self.est.shape[0]:
            rows = np.flatnonzero(self.used)
            need = int((self.nfr[rows] - 1).sum()) + m
            new = np.zeros((max(self.est.shape[0], 2 * need), 2))
            pos = 0
            for r in rows:  # compaction: rare, a copy per live stream
                k = int(self.nxt[r]) - 1  # estimates written so far
                new[pos:pos + k] = self.est[self.eoff[r]:self.eoff[r] + k]
                self.eoff[r] = pos
                pos += int(self.nfr[r]) - 1
            self.est, self.top = new, pos
        off = self.top
        self.top += m
        return off

    def add(self, sid, code, member, req, fs):
        if self.free:
            r = self.free.pop()
        else:
            if self.rows_top == self.cap:
                self._grow(2 * self.cap)
            r = self.rows_top
            self.rows_top += 1
        self.used[r] = True
        self.sid[r], self.code[r], self.member[r] = sid, code, member
        self.nxt[r], self.nfr[r] = 1, req.n_frames
        self.arr[r], self.fps[r] = req.arrival, req.fps
        self.due[r] = req.arrival + 1.0 / req.fps
        self.base[r], self.stride[r], self.pitch[r] = fs.base, fs.stride, fs.pitch
        self.npart[r] = req.params.n_particles
        self.eoff[r] = self._alloc_est(max(req.n_frames - 1, 0))
        return r

    def estimates_of(self, r):
        k = int(self.nxt[r]) - 1
        return self.est[self.eoff[r]:self.eoff[r] + k].copy()

    def remove(self, r):
        self.used[r] = False
        self.free.append(r)


@dataclass
class StreamResult:
    sid: int
    status: str          # "done", "rejected", "evicted", "failed"
    reason: str = ""
    admission_wait: float = float("nan")
    frames_done: int = 0
    estimates: list = field(default_factory=list)


class Scheduler:
    """Continuous-batching loop over a backend (see module docstring)."""

    def __init__(self, backend, clock=time.perf_counter, stall_timeout: float = 1.0,
                 stall_poll: float = 0.001):
        self.backend = backend
        self.clock = clock
        self.stall_timeout = stall_timeout
        self.stall_poll = stall_poll
        self.pending = []            # heap of (arrival, sid, request) not yet arrived
        self.queue = deque()         # arrived requests waiting for a slot
        self.due = []                # heap of (next frame's arrival, sid) of admitted streams
        self.live = {}               # sid -> _Live
        # FrameSeq streams step from columns when the backend has array calls
        self.cols = _Columns() if hasattr(backend, "step_arrays") else None
        self.results = {}            # sid -> StreamResult
        self.latencies = []          # per processed frame: ready - arrival (seconds)
        self.updates = 0             # particle updates done
        self.ticks = 0
        self.step_seconds = 0.0

    # -- submission ---------------------------------------------------------
    def submit(self, req: StreamRequest):
        reason = self.backend.validate(req.params)
        if reason:
            self.results[req.sid] = StreamResult(req.sid, "rejected", reason)
            return False
        heapq.heappush(self.pending, (req.arrival, req.sid, req))
        return True

    # -- one tick -----------------------------------------------------------
    def _arrivals(self, now):
        while self.pending and self.pending[0][0] <= now:
            _, _, req = heapq.heappop(self.pending)
            self.queue.append(req)

    def _admit(self, now):
        waiting = deque()
        while self.queue:
            req = self.queue.popleft()
            try:
                slot = self.backend.try_admit(req)
            except PfError as e:  # the pool cannot take streams any more
                self.results[req.sid] = StreamResult(req.sid, "failed", str(e), now - req.arrival)
                continue
            if slot is None:
                waiting.append(req)
                continue
            lv = _Live(req, slot, now)
            self.live[req.sid] = lv
            if self.cols is not None and isinstance(req.frame, FrameSeq) and req.n_frames > 1:
                code, member = self.backend.slot_code(slot)
                lv.row = self.cols.add(req.sid, code, member, req, req.frame)
            else:
                heapq.heappush(self.due, (req.arrival + 1.0 / req.fps, req.sid))
        self.queue = waiting

    def _finish(self, lv: _Live, status: str, reason: str = ""):
        self.backend.release(lv.slot)
        del self.live[lv.req.sid]
        if lv.row >= 0:
            lv.next_frame = int(self.cols.nxt[lv.row])
            lv.estimates = self.cols.estimates_of(lv.row)
            self.cols.remove(lv.row)
        self.results[lv.req.sid] = StreamResult(
            lv.req.sid, status, reason, lv.admitted - lv.req.arrival, lv.next_frame - 1, lv.estimates)

    def tick(self):
        """Admit, step every stream with a waiting frame once, record
        latencies, evict stalled streams.  Returns the number of frames
        stepped."""
        now = self.clock()
        self._arrivals(now)
        self._admit(now)
        # streams whose next frame has arrived, from the heap of due times
        work = []
        retry = []
        while self.due and self.due[0][0] <= now:
            _, sid = heapq.heappop(self.due)
            lv = self.live.get(sid)
            if lv is None:
                continue
            r = lv.req
            i = lv.next_frame
            if i >= r.n_frames:
                self._finish(lv, "done")
                continue
            t_arr = r.arrival + i / r.fps
            fr = r.frame(i)
            if fr is None:  # the source stalls: evict once it is late by the timeout
                if now - t_arr > self.stall_timeout:
                    self._finish(lv, "evicted", f"frame {i} late by more than {self.stall_timeout} s")
                else:
                    retry.append((now + self.stall_poll, sid))
                continue
            work.append((lv, fr, t_arr))
        for item in retry:
            heapq.heappush(self.due, item)
        if self.cols is not None:
            return self._step_arrays(work, now)
        if not work:
            return 0
        t0 = self.clock()
        failed = self.backend.step([(lv.slot, fr) for lv, fr, _ in work])
        ests = self.backend.estimates([lv.slot for lv, _, _ in work])
        done = self.clock()
        self.step_seconds += done - t0
        self.ticks += 1
        for (lv, _, t_arr), est in zip(work, ests):
            if lv.slot in failed:
                self._finish(lv, "failed", failed[lv.slot])
                continue
            self._advance(lv, est, done - t_arr)
        return len(work)

    def _advance(self, lv, est, latency):
        self.latencies.append(latency)
        self.updates += lv.req.params.n_particles
        lv.estimates.append(est)
        lv.next_frame += 1
        if lv.next_frame >= lv.req.n_frames:
            self._finish(lv, "done")
        else:
            heapq.heappush(self.due, (lv.req.arrival + lv.next_frame / lv.req.fps, lv.req.sid))

    def _step_arrays(self, work, now):
        """One tick through the backend's array calls: the heap's streams
        (`work`) and every FrameSeq stream whose next frame has arrived, in
        one batched step per pool."""
        c = self.cols
        rows = np.flatnonzero(c.used[:c.rows_top] & (c.due[:c.rows_top] <= now))
        ng = len(work)
        if ng == 0 and rows.size == 0:
            return 0
        codes = np.empty(ng + rows.size, dtype=np.int64)
        members = np.empty_like(codes)
        ptrs = np.empty_like(codes)
        pitches = np.empty_like(codes)
        for j, (lv, fr, _) in enumerate(work):
            codes[j], members[j] = self.backend.slot_code(lv.slot)
            if isinstance(fr, tuple):
                ptrs[j], pitches[j] = fr
            else:
                ptrs[j], pitches[j] = fr.data_ptr(), fr.stride(0)
        nx = c.nxt[rows]
        codes[ng:] = c.code[rows]
        members[ng:] = c.member[rows]
        ptrs[ng:] = c.base[rows] + nx * c.stride[rows]
        pitches[ng:] = c.pitch[rows]
        t0 = self.clock()
        failed = self.backend.step_arrays(codes, members, ptrs, pitches)  # {item index: reason}
        ests = self.backend.estimates_arrays(codes, members)
        done = self.clock()
        self.step_seconds += done - t0
        self.ticks += 1
        for j, (lv, _, t_arr) in enumerate(work):
            if j in failed:
                self._finish(lv, "failed", failed[j])
            else:
                self._advance(lv, tuple(ests[j]), done - t_arr)
        if rows.size:
            ok = np.ones(rows.size, dtype=bool)
            for j in failed:
                if j >= ng:
                    ok[j - ng] = False
            good, nxg = rows[ok], nx[ok]
            t_arr = c.arr[good] + nxg / c.fps[good]
            self.latencies.extend((done - t_arr).tolist())
            self.updates += int(c.npart[good].sum())
            c.est[c.eoff[good] + nxg - 1] = ests[ng:][ok]
            c.nxt[good] = nxg + 1
            c.due[good] = c.arr[good] + (nxg + 1) / c.fps[good]
            for j in np.flatnonzero(~ok):
                self._finish(self.live[int(c.sid[rows[j]])], "failed", failed[ng + int(j)])
            for r in good[nxg + 1 >= c.nfr[good]]:
                self._finish(self.live[int(c.sid[r])], "done")
        return ng + rows.size

    def idle(self):
        return not self.pending and not self.queue and not self.live

    def run(self, until: float = math.inf, sleep=time.sleep, poll: float = 0.0005):
        """Tick until every submitted stream has finished or the clock passes
        `until`."""
        while not self.idle() and self.clock() < until:
            if self.tick() == 0:
                sleep(poll)
        return self.summary()

    def summary(self, since_latency: int = 0):
        lat = np.array(self.latencies[since_latency:])
        st = {}
        for r in self.results.values():
            st[r.status] = st.get(r.status, 0) + 1
        waits = np.array([r.admission_wait for r in self.results.values()
                          if r.status in ("done", "evicted", "failed")])
        return dict(frames=int(lat.size),
                    latency_p50_ms=float(np.percentile(lat, 50) * 1e3) if lat.size else None,
                    latency_p99_ms=float(np.percentile(lat, 99) * 1e3) if lat.size else None,
                    admission_wait_p50_ms=float(np.percentile(waits, 50) * 1e3) if waits.size else None,
                    admission_wait_p99_ms=float(np.percentile(waits, 99) * 1e3) if waits.size else None,
                    streams=st, ticks=self.ticks, particle_updates=self.updates,
                    hbm_high_water_bytes=self.backend.high_water())


# ---------------------------------------------------------------------------
# GPU backend: one pf_batch per precision, slots in particle-count classes.

def slot_classes(n_min: int, n_max: int):
    """Particle capacities of the slot classes: powers of two covering
    [n_min, n_max]."""
    lo = 1 << max(0, math.ceil(math.log2(n_min)))
    caps = []
    c = lo
    while True:
        caps.append(c)
        if c >= n_max:
            break
        c *= 2
    return caps


def plan_pool(budget_bytes: int, dtype: str, caps, weights=None):
    """Slots per class for one precision so that the pool's workspace fits
    `budget_bytes`: counts proportional to `weights` (default equal)."""
    w = np.ones(len(caps)) if weights is None else np.asarray(weights, dtype=float)
    per = [pf_member_bytes(make_params(c, 64, 64, dtype)) for c in caps]
    scale = budget_bytes / float(np.dot(w, per))
    counts = [max(1, int(scale * wi)) for wi in w]
    return dict(zip(caps, counts))


class GpuPoolBackend:
    """Slot pools on one GPU: for every precision a pf_batch whose members are
    created at the class capacities and re-initialised for each stream."""

    def __init__(self, pools: dict, device="cuda:0", stream=None):
        """pools: {dtype name: {capacity: slots}}."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.batches = {}
        self.free = {}
        self.slot_cap = {}
        self.in_use_bytes = 0
        self.high = 0
        self.slot_bytes = {}
        for dt, classes in pools.items():
            params, caps = [], []
            for cap, count in sorted(classes.items()):
                for _ in range(count):
                    params.append(make_params(cap, 64, 64, dt))
                    caps.append(cap)
            b = Batch(params, device=device, stream=self.stream)
            self.batches[dt] = b
            n = len(params)
            self.free[dt] = {}
            for k, cap in enumerate(caps):
                self.free[dt].setdefault(cap, []).append(k)
                self.slot_cap[(dt, k)] = cap
                self.slot_bytes[(dt, k)] = pf_member_bytes(params[k])
            for cap in self.free[dt]:
                self.free[dt][cap].reverse()
            b._ptrs = np.zeros(n, dtype=np.uint64)
            b._pitch = np.zeros(n, dtype=np.int64)
            b._active = np.zeros(n, dtype=np.uint8)
        self.pool_bytes = sum(b.workspace.numel() for b in self.batches.values())

    @staticmethod
    def _dtype_name(code):
        return {PF_F64: "f64", PF_F32: "f32", PF_F16: "f16", PF_BF16: "bf16"}[code]

    def validate(self, params):
        try:
            pf_member_bytes(params)
        except PfError as e:
            return str(e)
        dt = self._dtype_name(params.dtype)
        if dt not in self.batches:
            return f"no pool for dtype {dt}"
        if params.n_particles > max(self.free[dt]):
            return f"n_particles {params.n_particles} above the largest slot class"
        return ""

    def try_admit(self, req):
        dt = self._dtype_name(req.params.dtype)
        for cap in sorted(self.free[dt]):
            if cap >= req.params.n_particles and self.free[dt][cap]:
                k = self.free[dt][cap].pop()
                self.batches[dt].reinit(k, req.params)
                self.in_use_bytes += self.slot_bytes[(dt, k)]
                self.high = max(self.high, self.in_use_bytes)
                return (dt, k)
        return None

    def release(self, slot):
        dt, k = slot
        self.free[dt][self.slot_cap[slot]].append(k)
        self.in_use_bytes -= self.slot_bytes[slot]

    def step(self, items):
        """items: [(slot, frame)] with frame an (H, W) uint8 device tensor or a
        (device pointer, row pitch) pair; one pf_batch_step per pool.  Returns
        {slot: error text} for the streams whose step failed."""
        by = {}
        for slot, fr in items:
            by.setdefault(slot[0], []).append((slot[1], fr))
        failed = {}
        for dt, lst in by.items():
            b = self.batches[dt]
            b._active[:] = 0
            for k, fr in lst:
                if isinstance(fr, tuple):  # (device pointer, row pitch)
                    b._ptrs[k], b._pitch[k] = fr
                else:                      # (H, W) uint8 tensor
                    b._ptrs[k] = fr.data_ptr()
                    b._pitch[k] = fr.stride(0)
                b._active[k] = 1
            try:
                b.step_ptrs(b._ptrs, b._pitch, b._active)
            except PfError as e:
                for k, _ in lst:
                    failed[(dt, k)] = str(e)
        return failed

    def estimates(self, slots):
        out = {}
        for dt in {s[0] for s in slots}:
            out[dt] = self.batches[dt].estimates()
        return [tuple(out[dt][k]) for dt, k in slots]

    # -- array calls: one column per item ------------------------------------
    _CODE = {"f64": PF_F64, "f32": PF_F32, "f16": PF_F16, "bf16": PF_BF16}

    def slot_code(self, slot):
        """(pool code, member) of a slot, for the array calls."""
        return self._CODE[slot[0]], slot[1]

    def step_arrays(self, codes, members, ptrs, pitches):
        """Step member members[j] of pool codes[j] on the frame at ptrs[j]
        (row pitch pitches[j]): one pf_batch_step per pool.  Returns {j:
        error text} for the items whose pool's step failed."""
        failed = {}
        for code in np.unique(codes):
            dt = self._dtype_name(int(code))
            b = self.batches[dt]
            m = codes == code
            ks = members[m]
            b._active[:] = 0
            b._active[ks] = 1
            b._ptrs[ks] = ptrs[m].astype(np.uint64)
            b._pitch[ks] = pitches[m]
            try:
                b.step_ptrs(b._ptrs, b._pitch, b._active)
            except PfError as e:
                for j in np.flatnonzero(m):
                    failed[int(j)] = str(e)
        return failed

    def estimates_arrays(self, codes, members):
        """The latest estimates of the items, as an (items, 2) array."""
        out = np.empty((codes.size, 2))
        for code in np.unique(codes):
            m = codes == code
            out[m] = self.batches[self._dtype_name(int(code))].estimates()[members[m]]
        return out

    def high_water(self):
        return self.high

    def close(self):
        for b in self.batches.values():
            b.close()


# ---------------------------------------------------------------------------
# Byte-budget admission.

class ByteArena:
    """First-fit allocator of byte ranges of [0, size), each 256-byte aligned;
    a freed range merges with free neighbours.  Offsets only: the caller maps
    them onto its device memory."""

    def __init__(self, size: int):
        self.size = size - size % WS_ALIGN
        self.starts = [0] if self.size else []   # free ranges, sorted by start
        self.lens = [self.size] if self.size else []
        self.used = 0
        self.high = 0

    @staticmethod
    def rounded(nbytes: int) -> int:
        return -(-int(nbytes) // WS_ALIGN) * WS_ALIGN

    def alloc(self, nbytes: int):
        """Offset of a free range of nbytes (rounded up to 256), or None."""
        need = self.rounded(nbytes)
        for i, ln in enumerate(self.lens):
            if ln >= need:
                off = self.starts[i]
                if ln == need:
                    del self.starts[i], self.lens[i]
                else:
                    self.starts[i] += need
                    self.lens[i] -= need
                self.used += need
                self.high = max(self.high, self.used)
                return off
        return None

    def release(self, off: int, nbytes: int):
        need = self.rounded(nbytes)
        i = bisect.bisect_left(self.starts, off)
        if (i < len(self.starts) and self.starts[i] < off + need) or \
                (i > 0 and self.starts[i - 1] + self.lens[i - 1] > off):
            raise ValueError(f"range [{off}, {off + need}) overlaps a free range")
        self.starts.insert(i, off)
        self.lens.insert(i, need)
        if i + 1 < len(self.starts) and off + need == self.starts[i + 1]:  # merge the next
            self.lens[i] += self.lens[i + 1]
            del self.starts[i + 1], self.lens[i + 1]
        if i > 0 and self.starts[i - 1] + self.lens[i - 1] == off:  # merge into the previous
            self.lens[i - 1] += self.lens[i]
            del self.starts[i], self.lens[i]
        self.used -= need

    def largest_free(self) -> int:
        return max(self.lens, default=0)


class GpuByteBackend(GpuPoolBackend):
    """One pf_batch per precision with `handles` members and, for the
    precision's HBM budget, a device arena from which every admitted stream
    gets exactly its workspace bytes; the member is rebound to that share
    (pf_batch_rebind).  A released member is left as it is (it is not
    stepped again, and its stale block is only read by the estimates'
    gather, from the arena), so a release costs no device work; its tiles
    still count against the batch's plan, which holds `plan_factor` times
    the arena's worth of tiles plus one per member.  When an admission would
    still overflow the plan, the idle members holding the most tiles are
    first parked on one-particle filters on small shares of their own.
    Free members are taken largest-stale-first, so a rebind also retires
    the most stale tiles."""

    def __init__(self, budgets: dict, handles: dict, device="cuda:0", stream=None, plan_factor: float = 2.0):
        """budgets: {dtype name: arena bytes}; handles: {dtype name: members}."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.batches, self.arenas, self.arena_mem, self.park_mem = {}, {}, {}, {}
        self.share = {}
        self.tiny = {}
        self.free_heap = {}                    # (-stale tiles, member) of the free members
        self.cur_tiles, self.tiles_used, self.tiles_cap = {}, {}, {}
        self.parked = 0                        # members parked to make room in a plan
        for dt, budget in budgets.items():
            m = int(handles[dt])
            tiny = make_params(1, 64, 64, dt)
            tiny_bytes = ByteArena.rounded(pf_member_bytes(tiny))
            # tiles the arena's bytes can hold at most
            per_tile = pf_member_bytes(make_params(1 << 20, 64, 64, dt)) / 1024.0
            cap = int(plan_factor * (budget // per_tile)) + m
            b = Batch([tiny] * m, device=device, stream=self.stream, max_tiles=cap)
            b._ptrs = np.zeros(m, dtype=np.uint64)
            b._pitch = np.zeros(m, dtype=np.int64)
            b._active = np.zeros(m, dtype=np.uint8)
            self.batches[dt] = b
            self.arenas[dt] = ByteArena(int(budget))
            self.arena_mem[dt] = torch.empty(self.arenas[dt].size, dtype=torch.uint8, device=self.device)
            self.park_mem[dt] = torch.empty(m * tiny_bytes, dtype=torch.uint8, device=self.device)
            self.tiny[dt] = (tiny, tiny_bytes)
            self.free_heap[dt] = [(-1, k) for k in range(m)]
            heapq.heapify(self.free_heap[dt])
            self.cur_tiles[dt] = [1] * m
            self.tiles_used[dt] = m
            self.tiles_cap[dt] = cap
        self.pool_bytes = sum(b.workspace.numel() for b in self.batches.values()) + \
            sum(t.numel() for t in self.arena_mem.values()) + sum(t.numel() for t in self.park_mem.values())

    def _park(self, dt, excess):
        """Park free members, most tiles first, until `excess` plan tiles are
        freed; returns what is still missing."""
        tiny, tiny_bytes = self.tiny[dt]
        heap, cur = self.free_heap[dt], self.cur_tiles[dt]
        parked = []
        while excess > 0 and heap and -heap[0][0] > 1:
            _, j = heapq.heappop(heap)
            self.batches[dt].rebind(j, tiny, self.park_mem[dt].data_ptr() + j * tiny_bytes, tiny_bytes)
            excess -= cur[j] - 1
            self.tiles_used[dt] -= cur[j] - 1
            cur[j] = 1
            parked.append(j)
            self.parked += 1
        for j in parked:
            heapq.heappush(heap, (-1, j))
        return excess

    def validate(self, params):
        try:
            need = pf_member_bytes(params)
        except PfError as e:
            return str(e)
        dt = self._dtype_name(params.dtype)
        if dt not in self.batches:
            return f"no pool for dtype {dt}"
        if ByteArena.rounded(need) > self.arenas[dt].size:
            return f"workspace of {need} bytes above the {dt} pool's budget of {self.arenas[dt].size}"
        return ""

    def try_admit(self, req):
        dt = self._dtype_name(req.params.dtype)
        heap = self.free_heap[dt]
        if not heap:
            return None
        need = pf_member_bytes(req.params)
        off = self.arenas[dt].alloc(need)
        if off is None:
            return None
        _, k = heapq.heappop(heap)
        cur = self.cur_tiles[dt]
        new_t = -(-int(req.params.n_particles) // 1024)
        try:
            # room in the plan: the member's stale tiles go, the stream's come
            excess = self.tiles_used[dt] - cur[k] + new_t - self.tiles_cap[dt]
            if excess > 0 and self._park(dt, excess) > 0:
                self.arenas[dt].release(off, need)
                heapq.heappush(heap, (-cur[k], k))
                return None
            self.batches[dt].rebind(k, req.params, self.arena_mem[dt].data_ptr() + off,
                                    ByteArena.rounded(need))
        except PfError:
            self.arenas[dt].release(off, need)
            heapq.heappush(heap, (-cur[k], k))
            raise
        self.tiles_used[dt] += new_t - cur[k]
        cur[k] = new_t
        self.share[(dt, k)] = (off, need)
        return (dt, k)

    def release(self, slot):
        dt, k = slot
        off, need = self.share.pop(slot)
        self.arenas[dt].release(off, need)
        heapq.heappush(self.free_heap[dt], (-self.cur_tiles[dt][k], k))

    def high_water(self):
        return sum(a.high for a in self.arenas.values())

    def in_use(self):
        return sum(a.used for a in self.arenas.values())
