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
