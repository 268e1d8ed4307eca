"""Host backend for testing the serving scheduler on the CPU: every slot is a
filter stepped by the FP64 oracle, on a virtual clock."""
from __future__ import annotations

import numpy as np

import oracle
import paper_2308_00763_amd as pf


class VirtualClock:
    def __init__(self, t=0.0):
        self.t = t

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """caps: {capacity: slots}.  fail_on: {sid: frame index whose step fails}.
    step_cost: seconds the virtual clock advances per batched step."""

    def __init__(self, caps, clock, fail_on=None, step_cost=0.002):
        self.free = {c: list(range(n))[::-1] for c, n in caps.items()}
        self.clock = clock
        self.fail_on = dict(fail_on or {})
        self.step_cost = step_cost
        self.state = {}
        self.in_use = 0
        self.high = 0
        self.steps = 0

    def validate(self, params):
        try:
            pf.pf_workspace_bytes(params)
        except pf.PfError as e:
            return str(e)
        if params.n_particles > max(self.free):
            return "n_particles above the largest slot class"
        return ""

    def try_admit(self, req):
        p = req.params
        for cap in sorted(self.free):
            if cap >= p.n_particles and self.free[cap]:
                slot = (cap, self.free[cap].pop(), req.sid)
                op = oracle.make_params(p.n_particles, p.width, p.height, radius=p.disk_radius,
                                        drift=(p.drift_x, p.drift_y), sigma=(p.sigma_x, p.sigma_y),
                                        seed=p.seed, stream_id=p.stream_id)
                self.state[slot] = dict(op=op, x=np.full(p.n_particles, p.x0),
                                        y=np.full(p.n_particles, p.y0), t=0, est=(p.x0, p.y0))
                self.in_use += cap
                self.high = max(self.high, self.in_use)
                return slot
        return None

    def release(self, slot):
        cap, k, _ = slot
        self.free[cap].append(k)
        del self.state[slot]
        self.in_use -= cap

    def step(self, items):
        self.steps += 1
        failed = {}
        for slot, frame in items:
            st = self.state[slot]
            if self.fail_on.get(slot[2]) == st["t"] + 1:
                failed[slot] = "injected step failure"
                continue
            out = oracle.step(st["op"], st["t"] + 1, frame, st["x"], st["y"])
            st.update(x=out["x"], y=out["y"], t=st["t"] + 1, est=tuple(out["est"]))
        self.clock.t += self.step_cost
        return failed

    def estimates(self, slots):
        return [self.state[s]["est"] if s in self.state else (np.nan, np.nan) for s in slots]

    def high_water(self):
        return self.high


class ArrayFakeBackend(FakeBackend):
    """FakeBackend with the array calls of the GPU backends, for FrameSeq
    streams: a frame "pointer" is stream_key << 32 | i << 20, resolved to
    frame i of the host video registered under that key."""

    STRIDE = 1 << 20

    def __init__(self, caps, clock, fail_on=None, step_cost=0.002):
        super().__init__(caps, clock, fail_on=fail_on, step_cost=step_cost)
        self.videos = {}      # key -> (T, H, W) frames
        self.ids = {}         # member id -> slot
        self.next_id = 0
        self.array_steps = 0

    def frame_seq(self, key, frames):
        from paper_2308_00763_amd.serve import FrameSeq
        self.videos[key] = frames
        return FrameSeq(key << 32, self.STRIDE, frames.shape[2])

    def slot_code(self, slot):
        for k, s in self.ids.items():
            if s == slot:
                return 0, k
        self.ids[self.next_id] = slot
        self.next_id += 1
        return 0, self.next_id - 1

    def release(self, slot):
        self.ids = {k: s for k, s in self.ids.items() if s != slot}
        super().release(slot)

    def _frame(self, ptr):
        key = int(ptr) >> 32
        return self.videos[key][(int(ptr) - (key << 32)) // self.STRIDE]

    def step_arrays(self, codes, members, ptrs, pitches):
        """Every item is a FrameSeq stream's frame (the tests give this
        backend no other kind)."""
        self.array_steps += 1
        slots = [self.ids[int(k)] for k in members]
        assert all(int(q) == self.videos[int(p) >> 32].shape[2] for p, q in zip(ptrs, pitches))
        failed = self.step([(s, self._frame(p)) for s, p in zip(slots, ptrs)])
        return {j: failed[s] for j, s in enumerate(slots) if s in failed}

    def estimates_arrays(self, codes, members):
        return np.array(self.estimates([self.ids[int(k)] for k in members]), dtype=float)
