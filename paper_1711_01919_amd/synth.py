"""Seeded synthetic inputs: frames, bin counts and query rectangles.

This module only draws inputs.  It holds none of the integral-histogram
arithmetic (no binning, no scans, no queries), so both the HIP path and the
CPU oracle can be fed from it without sharing any of the method.

The paper measures on image sequences it does not name or ship (HD video,
640x480 and 512x512 frames, an 8k x 8k image); the generators below stand in
for them with the same shapes, bin counts and value ranges.  Every draw uses
``numpy.random.default_rng(seed)`` (PCG64) in the order written here.

Workloads:
  plain_frame()        640x480 uniform pixels, B=32, 1000 rectangles  (seed 0)
  disc_sequence()      64 frames 1920x1080, gradient + noise + 8 moving
                       bright discs, B=64                               (seed 1)
  mixture_frame()      8192x8192, 8-level Gaussian mixture, B=128,
                       1e6 rectangles                                   (seed 2)
  uneven_batch()       256 frames of mixed resolution and bin count     (seed 3)
  stream_plan()        16 video streams with Poisson arrivals           (seed 5)
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

RESOLUTIONS_UNEVEN = [(240, 320), (480, 640), (720, 1280), (1080, 1920), (2160, 3840)]  # (H, W)
BINS_UNEVEN = [16, 32, 64, 128]
RESOLUTIONS_STREAM = [(480, 640), (720, 1280), (1080, 1920), (1440, 2560), (2160, 3840)]
BINS_STREAM = [32, 64]


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def uniform_frame(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    return rng.integers(0, 256, size=(H, W), dtype=np.uint8)


def random_rects(rng: np.random.Generator, H: int, W: int, n: int) -> np.ndarray:
    """n rectangles {x0, y0, x1, y1} with inclusive corners: two columns drawn
    uniformly in [0, W) and sorted, then two rows in [0, H) sorted."""
    xs = np.sort(rng.integers(0, W, size=(n, 2)), axis=1)
    ys = np.sort(rng.integers(0, H, size=(n, 2)), axis=1)
    r = np.empty((n, 4), dtype=np.int32)
    r[:, 0] = xs[:, 0]
    r[:, 1] = ys[:, 0]
    r[:, 2] = xs[:, 1]
    r[:, 3] = ys[:, 1]
    return r


# ---------------------------------------------------------------------------
# 640x480, B=32 (the paper's headline frame size and bin count)
# ---------------------------------------------------------------------------
def plain_frame(seed: int = 0, H: int = 480, W: int = 640, B: int = 32, n_rects: int = 1000):
    rng = np.random.default_rng(seed)
    I = uniform_frame(rng, H, W)
    rects = random_rects(rng, H, W, n_rects)
    return I, B, rects


# ---------------------------------------------------------------------------
# moving-disc video frames (HD sequences of the dual-buffering experiment)
# ---------------------------------------------------------------------------
@dataclass
class DiscScene:
    H: int
    W: int
    cx: np.ndarray
    cy: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    r: np.ndarray
    value: int = 230
    sigma: float = 12.0
    speed: float = 5.0

    @staticmethod
    def new(rng: np.random.Generator, H: int, W: int, n_discs: int = 8, speed: float = 5.0):
        r = rng.integers(20, 81, size=n_discs).astype(np.float64)
        cx = rng.uniform(0, W, size=n_discs)
        cy = rng.uniform(0, H, size=n_discs)
        th = rng.uniform(0, 2 * np.pi, size=n_discs)
        return DiscScene(H, W, cx, cy, speed * np.cos(th), speed * np.sin(th), r, speed=speed)

    def render(self, rng: np.random.Generator) -> np.ndarray:
        H, W = self.H, self.W
        xs = np.arange(W, dtype=np.float64)
        ys = np.arange(H, dtype=np.float64)
        img = 64.0 + 128.0 * (xs[None, :] / W + ys[:, None] / H) / 2.0
        img = img + rng.normal(0.0, self.sigma, size=(H, W))
        for k in range(len(self.r)):
            x0 = max(0, int(self.cx[k] - self.r[k])); x1 = min(W, int(self.cx[k] + self.r[k]) + 1)
            y0 = max(0, int(self.cy[k] - self.r[k])); y1 = min(H, int(self.cy[k] + self.r[k]) + 1)
            if x0 >= x1 or y0 >= y1:
                continue
            dx = xs[x0:x1][None, :] - self.cx[k]
            dy = ys[y0:y1][:, None] - self.cy[k]
            m = dx * dx + dy * dy <= self.r[k] * self.r[k]
            img[y0:y1, x0:x1][m] = self.value
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)

    def step(self):
        """Advance every disc by its velocity, reflecting at the borders."""
        self.cx += self.vx
        self.cy += self.vy
        for c, v, lim in ((self.cx, self.vx, self.W), (self.cy, self.vy, self.H)):
            lo = c < 0
            c[lo] = -c[lo]; v[lo] = -v[lo]
            hi = c > lim - 1
            c[hi] = 2 * (lim - 1) - c[hi]; v[hi] = -v[hi]


def disc_sequence(seed: int = 1, n_frames: int = 64, H: int = 1080, W: int = 1920, B: int = 64):
    """n_frames uint8 frames (n, H, W) of a gradient + N(0,12^2) noise + 8 moving
    discs (radius 20..80 px, value 230, 5 px per frame, reflecting)."""
    rng = np.random.default_rng(seed)
    scene = DiscScene.new(rng, H, W)
    frames = np.empty((n_frames, H, W), dtype=np.uint8)
    for f in range(n_frames):
        frames[f] = scene.render(rng)
        scene.step()
    return frames, B


# ---------------------------------------------------------------------------
# 8192x8192 mixture-of-Gaussians frame (the multi-GPU experiment's 64 MB image)
# ---------------------------------------------------------------------------
def mixture_frame(seed: int = 2, H: int = 8192, W: int = 8192, B: int = 128,
                  n_rects: int = 1_000_000, sigma: float = 10.0):
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, 8, size=(H, W), dtype=np.uint8)
    means = 16.0 + 32.0 * np.arange(8)
    I = np.empty((H, W), dtype=np.uint8)
    step = max(1, (1 << 24) // W)                       # fill in row blocks to bound temporaries
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        v = means[comp[y0:y1]] + rng.normal(0.0, sigma, size=(y1 - y0, W))
        I[y0:y1] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    rects = random_rects(rng, H, W, n_rects)
    return I, B, rects


# ---------------------------------------------------------------------------
# 256 frames of uneven resolution and bin count
# ---------------------------------------------------------------------------
@dataclass
class UnevenBatch:
    frames: list = field(default_factory=list)   # list of (H, W) uint8 arrays
    bins: list = field(default_factory=list)     # list of int

    @property
    def entries(self) -> int:
        return int(sum(f.shape[0] * f.shape[1] * b for f, b in zip(self.frames, self.bins)))


def uneven_batch(seed: int = 3, n_frames: int = 256, scale: int = 1) -> UnevenBatch:
    """Resolution index and bin index drawn first (uniform over the lists
    above), then the uniform pixels frame by frame.  ``scale`` > 1 divides
    every side by it (small variant for tests)."""
    rng = np.random.default_rng(seed)
    ri = rng.integers(0, len(RESOLUTIONS_UNEVEN), size=n_frames)
    bi = rng.integers(0, len(BINS_UNEVEN), size=n_frames)
    ub = UnevenBatch()
    for k in range(n_frames):
        H, W = RESOLUTIONS_UNEVEN[ri[k]]
        H = max(1, H // scale); W = max(1, W // scale)
        ub.frames.append(uniform_frame(rng, H, W))
        ub.bins.append(BINS_UNEVEN[bi[k]])
    return ub


# ---------------------------------------------------------------------------
# 16 video streams for the serving loop
# ---------------------------------------------------------------------------
@dataclass
class StreamSpec:
    H: int
    W: int
    B: int
    fps: float
    arrivals: np.ndarray     # seconds from start


def stream_plan(seed: int = 5, n_streams: int = 16, duration_s: float = 10.0,
                fps_lo: float = 30.0, fps_hi: float = 120.0):
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(n_streams):
        H, W = RESOLUTIONS_STREAM[int(rng.integers(0, len(RESOLUTIONS_STREAM)))]
        B = BINS_STREAM[int(rng.integers(0, len(BINS_STREAM)))]
        fps = float(rng.uniform(fps_lo, fps_hi))
        t, arr = 0.0, []
        while True:
            t += float(rng.exponential(1.0 / fps))
            if t >= duration_s:
                break
            arr.append(t)
        specs.append(StreamSpec(H, W, B, fps, np.asarray(arr)))
    return specs


def stream_frame_pool(seed: int, spec: StreamSpec, pool: int = 4, n_rects: int = 256):
    """A small pool of disc frames (and a rectangle set per frame) that a
    stream cycles through; generated before any timing starts."""
    rng = np.random.default_rng(seed)
    scene = DiscScene.new(rng, spec.H, spec.W)
    frames, rects = [], []
    for _ in range(pool):
        frames.append(scene.render(rng))
        rects.append(random_rects(rng, spec.H, spec.W, n_rects))
        scene.step()
    return frames, rects
