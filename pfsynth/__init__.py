"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs: greyscale videos of a disk moving over a flat
background with Gaussian pixel noise, shaped like the paper's tracking workload
(arXiv:2308.00763, Sec. 5, verification paragraph: a circular object moving in
the plane, one foreground and one background intensity, added Gaussian noise,
bouncing specularly off a wall).  It holds none of the particle filter's
arithmetic and is imported by both the oracle-side tests and the GPU side.

Conventions: x is the column, y is the row; frames are (H, W) uint8, row-major.
The object at frame t is drawn at an integer centre; a pixel (i, j) is
foreground when (j - cx)^2 + (i - cy)^2 < r^2.  Noise N(0, sigma^2) is added,
rounded half up and clipped to [0, 255].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Video:
    frames: np.ndarray      # (T, H, W) uint8
    centres: np.ndarray     # (T, 2) float64, ground-truth (x, y) per frame
    radius: int
    noise_sigma: float


def _reflect(p: int, v: int, lo: int, hi: int):
    """Advance p by v inside [lo, hi], reflecting specularly off both walls."""
    p = p + v
    while p < lo or p > hi:
        if p < lo:
            p = 2 * lo - p
            v = -v
        if p > hi:
            p = 2 * hi - p
            v = -v
    return p, v


def trajectory(T: int, start, velocity, width: int, height: int, radius: int,
               bounce: bool = False) -> np.ndarray:
    """Integer object centres for frames 0..T-1 (constant velocity, optional bounce)."""
    cx, cy = int(start[0]), int(start[1])
    vx, vy = int(velocity[0]), int(velocity[1])
    out = np.zeros((T, 2), dtype=np.float64)
    for t in range(T):
        out[t] = (cx, cy)
        if bounce:
            cx, vx = _reflect(cx, vx, radius, width - 1 - radius)
            cy, vy = _reflect(cy, vy, radius, height - 1 - radius)
        else:
            cx, cy = cx + vx, cy + vy
    return out


def render(width: int, height: int, centres: np.ndarray, radius: int, noise_sigma: float,
           seed: int, fg: int = 228, bg: int = 100) -> np.ndarray:
    """Draw the frames for the given centres with PCG64(seed) noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = centres.shape[0]
    video = np.empty((T, height, width), dtype=np.uint8)
    r2 = radius * radius
    for t in range(T):
        cx, cy = int(centres[t, 0]), int(centres[t, 1])
        img = np.full((height, width), float(bg), dtype=np.float32)
        y0, y1 = max(cy - radius, 0), min(cy + radius, height - 1)
        x0, x1 = max(cx - radius, 0), min(cx + radius, width - 1)
        if y0 <= y1 and x0 <= x1:
            jj, ii = np.meshgrid(np.arange(x0, x1 + 1), np.arange(y0, y1 + 1))
            inside = (jj - cx) ** 2 + (ii - cy) ** 2 < r2
            sub = img[y0:y1 + 1, x0:x1 + 1]
            sub[inside] = float(fg)
        if noise_sigma > 0:
            img += rng.standard_normal((height, width), dtype=np.float32) * np.float32(noise_sigma)
        video[t] = np.clip(np.floor(img + np.float32(0.5)), 0, 255).astype(np.uint8)
    return video


def moving_disk(width: int, height: int, T: int, radius: int, start, velocity,
                noise_sigma: float, seed: int, bounce: bool = False,
                fg: int = 228, bg: int = 100) -> Video:
    centres = trajectory(T, start, velocity, width, height, radius, bounce)
    frames = render(width, height, centres, radius, noise_sigma, seed, fg, bg)
    return Video(frames, centres, radius, float(noise_sigma))


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the paper's tracking workload scaled to the
# configurations this library is measured on.

@dataclass
class Workload:
    name: str
    width: int
    height: int
    frames: int
    radius: int
    noise_sigma: float
    n_particles: int
    start: tuple
    velocity: tuple
    filter_seed: int
    video_seed: int
    drift: tuple = (1.0, -2.0)
    sigma: tuple = (5.0, 2.0)


WORKLOADS = {
    # single filter, 128x128, 10 frames, r=5, N=1000 (parity case)
    "disk128_n1000": Workload("disk128_n1000", 128, 128, 10, 5, 2.0, 1000,
                              (64, 64), (1, -2), 0, 1),
    # precision sweep: 1024x1024, 100 frames, r=5, N=2^20
    "disk1024_n1m": Workload("disk1024_n1m", 1024, 1024, 100, 5, 2.0, 1 << 20,
                             (512, 512), (1, -2), 0, 2),
    # large-N stress: 512x512, 50 frames, r=8, noise sigma 8, N=2^24
    "disk512_r8_n16m": Workload("disk512_r8_n16m", 512, 512, 50, 8, 8.0, 1 << 24,
                                (256, 256), (1, -2), 0, 3),
    # the paper's accuracy video: 512x512, 100 frames, the object moving at
    # the motion model's drift (+1, -2) toward y = 0, bouncing off it at frame
    # 47 (the disk touches the wall; the y velocity flips), tracked with 128
    # particles
    "bounce512_n128": Workload("bounce512_n128", 512, 512, 100, 5, 2.0, 128,
                               (200, 100), (1, -2), 0, 7),
}


def workload_video(w: Workload, frames: int | None = None, bounce: bool = False) -> Video:
    T = w.frames if frames is None else frames
    return moving_disk(w.width, w.height, T, w.radius, w.start, w.velocity, w.noise_sigma,
                       w.video_seed, bounce=bounce)


# ---------------------------------------------------------------------------
# Fleets of independent streams (many trackers advanced together): each stream
# has its own video of the disk moving at an integer velocity without bouncing,
# its own particle count and noise level.

@dataclass
class Stream:
    stream_id: int
    n_particles: int
    start: tuple
    velocity: tuple
    noise_sigma: float
    video_seed: int


def stream_mix(n_streams: int, side: int = 256, frames: int = 50, radius: int = 5,
               n_lo: int = 256, n_hi: int = 65536, noise=(2.0, 6.0), vmax: int = 3,
               seed: int = 4_000_000) -> list:
    """Parameters of n_streams streams: N log-uniform in [n_lo, n_hi] (rounded),
    velocity uniform in {-vmax..vmax}^2, noise sigma uniform in `noise`, start
    uniform among the centres that keep the disk inside [r, side-1-r] for all
    frames.  Stream i has stream_id i and video seed seed + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    span = frames - 1
    for i in range(n_streams):
        n = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        n = min(max(n, n_lo), n_hi)
        v = (int(rng.integers(-vmax, vmax + 1)), int(rng.integers(-vmax, vmax + 1)))
        start = []
        for c in range(2):
            lo = radius - min(0, v[c] * span)
            hi = side - 1 - radius - max(0, v[c] * span)
            start.append(int(rng.integers(lo, hi + 1)))
        sig = float(rng.uniform(noise[0], noise[1]))
        out.append(Stream(i, n, (start[0], start[1]), v, sig, seed + i))
    return out


def stream_video(s: Stream, side: int, frames: int, radius: int = 5) -> Video:
    """The stream's own video, drawn on the host with PCG64(video_seed)."""
    return moving_disk(side, side, frames, radius, s.start, s.velocity, s.noise_sigma,
                       s.video_seed)


def render_fleet_torch(streams, t: int, side: int, radius: int, device, seed: int,
                       fg: int = 228, bg: int = 100):
    """Frame t of every stream as one (n, side, side) uint8 tensor drawn on
    `device`: same scene and noise model as stream_video, but the noise comes
    from torch's generator seeded with seed + t (for fleets whose videos are
    too large to draw on the host)."""
    import torch
    n = len(streams)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) + int(t))
    c = torch.tensor([[s.start[0] + s.velocity[0] * t, s.start[1] + s.velocity[1] * t]
                      for s in streams], dtype=torch.float32, device=device)
    sig = torch.tensor([s.noise_sigma for s in streams], dtype=torch.float32, device=device)
    ax = torch.arange(side, dtype=torch.float32, device=device)
    dx2 = (ax.view(1, 1, side) - c[:, 0].view(n, 1, 1)) ** 2
    dy2 = (ax.view(1, side, 1) - c[:, 1].view(n, 1, 1)) ** 2
    img = torch.where(dx2 + dy2 < float(radius * radius), float(fg), float(bg))
    img = img + torch.randn((n, side, side), generator=g, device=device) * sig.view(n, 1, 1)
    return torch.clamp(torch.floor(img + 0.5), 0, 255).to(torch.uint8)


def render_video_torch(centres, side: int, radius: int, noise_sigma: float, device, seed: int,
                       fg: int = 228, bg: int = 100, chunk: int = 32):
    """A (T, side, side) uint8 video drawn on `device` for the given integer
    centres (T, 2): the scene and noise model of `render`, with the noise
    from torch's generator seeded with `seed`."""
    import torch
    T = len(centres)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((T, side, side), dtype=torch.uint8, device=device)
    c = torch.as_tensor(np.asarray(centres, dtype=np.float32), device=device)
    ax = torch.arange(side, dtype=torch.float32, device=device)
    for t0 in range(0, T, chunk):
        cc = c[t0:t0 + chunk]
        m = cc.shape[0]
        dx2 = (ax.view(1, 1, side) - cc[:, 0].view(m, 1, 1)) ** 2
        dy2 = (ax.view(1, side, 1) - cc[:, 1].view(m, 1, 1)) ** 2
        img = torch.where(dx2 + dy2 < float(radius * radius), float(fg), float(bg))
        img = img + torch.randn((m, side, side), generator=g, device=device) * float(noise_sigma)
        out[t0:t0 + m] = torch.clamp(torch.floor(img + 0.5), 0, 255).to(torch.uint8)
    return out
