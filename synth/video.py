"""Seeded synthetic video streams for the pROST workloads.

This module only draws inputs: planted low-rank backgrounds, moving
foreground objects, additive noise and random orthonormal starting bases.
It holds none of the tracker's arithmetic and is shared by the tests, the
benchmark and the smoke check on both sides of every comparison.

Reproducibility: per-stream constants come from
``numpy.random.default_rng([seed, stream])`` and everything drawn for frame
n from ``default_rng([seed, stream, n])``, so any frame can be regenerated
on its own.

Layout: a frame is planar, all P = H*W pixels of channel 0 first, each
plane row-major (pixel p = row*W + col, entry e = c*P + p).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def random_orthonormal(m, k, rng):
    """m x k matrix with orthonormal columns: reduced QR of a Gaussian matrix,
    signs fixed so that diag(R) > 0."""
    G = rng.standard_normal((m, k))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def initial_subspace(m, k, seed, stream=0):
    """Random starting basis U0 (a reduced QR of a random m x k matrix)."""
    rng = np.random.default_rng([int(seed), int(stream), 0x5EED])
    return random_orthonormal(m, k, rng)


def _bounce(p0, v, n, lo, hi):
    """Position at frame n of a point moving with velocity v that reflects
    at lo and hi (closed form triangle wave)."""
    span = hi - lo
    if span <= 0:
        return lo
    q = (p0 - lo + v * n) % (2 * span)
    return lo + (q if q <= span else 2 * span - q)


@dataclasses.dataclass
class VideoSpec:
    width: int
    height: int
    channels: int
    rank: int
    seed: int
    stream: int = 0
    noise: float = 0.01
    fg_kind: str = "rects"          # "rects" | "ellipses" | "none"
    fg_count: int = 3
    fg_density: float = 0.05        # fraction of pixels covered (approx.)
    speed: tuple = (1.0, 2.0)       # px / frame
    jitter: int = 0                 # camera shake: integer shift in [-j, j]
    period: tuple = (50.0, 200.0)   # background coefficient periods (frames)

    @property
    def P(self):
        return self.width * self.height

    @property
    def m(self):
        return self.channels * self.P


class SyntheticVideo:
    """Frame source: background Q c(n) on a (possibly padded) canvas, cropped
    at a per-frame jitter offset, occluded by moving objects textured with
    U[0,1] values, plus N(0, noise^2) on every entry."""

    def __init__(self, spec: VideoSpec):
        self.spec = spec
        s = spec
        rng = np.random.default_rng([s.seed, s.stream])
        j = s.jitter
        self.cw, self.ch = s.width + 2 * j, s.height + 2 * j
        mc = s.channels * self.cw * self.ch
        self.Q = random_orthonormal(mc, s.rank, rng)
        self.T = rng.uniform(s.period[0], s.period[1], size=s.rank)
        self.ph = rng.uniform(0.0, 2.0 * math.pi, size=s.rank)
        self.objects = []
        if s.fg_kind != "none" and s.fg_count > 0:
            area = s.fg_density * s.P / s.fg_count
            for _ in range(s.fg_count):
                aspect = rng.uniform(0.6, 1.6)
                bw = max(1, int(round(math.sqrt(area * aspect))))
                bh = max(1, int(round(area / bw)))
                if s.fg_kind == "ellipses":   # area pi a b = area -> scale box
                    bw = max(1, int(round(bw * 2 / math.sqrt(math.pi))))
                    bh = max(1, int(round(bh * 2 / math.sqrt(math.pi))))
                bw, bh = min(bw, s.width), min(bh, s.height)
                speed = rng.uniform(s.speed[0], s.speed[1])
                ang = rng.uniform(0.0, 2.0 * math.pi)
                obj = dict(w=bw, h=bh,
                           x0=rng.uniform(0, s.width - bw), y0=rng.uniform(0, s.height - bh),
                           vx=speed * math.cos(ang), vy=speed * math.sin(ang),
                           tex=rng.uniform(0.0, 1.0, size=(s.channels, bh, bw)))
                if s.fg_kind == "ellipses":
                    yy, xx = np.mgrid[0:bh, 0:bw]
                    cy, cx = (bh - 1) / 2.0, (bw - 1) / 2.0
                    obj["shape"] = (((yy - cy) / max(bh / 2.0, 0.5)) ** 2 +
                                    ((xx - cx) / max(bw / 2.0, 0.5)) ** 2) <= 1.0
                else:
                    obj["shape"] = np.ones((bh, bw), bool)
                self.objects.append(obj)

    def coeffs(self, n):
        """Smooth background coefficients in [0, 1]."""
        return 0.5 + 0.5 * np.sin(2.0 * math.pi * n / self.T + self.ph)

    def frame(self, n, with_mask=False):
        s = self.spec
        rng = np.random.default_rng([s.seed, s.stream, int(n)])
        bg = (self.Q @ self.coeffs(n)).reshape(s.channels, self.ch, self.cw)
        if s.jitter:
            dx, dy = rng.integers(-s.jitter, s.jitter + 1, size=2)
            oy, ox = s.jitter + dy, s.jitter + dx
            img = bg[:, oy:oy + s.height, ox:ox + s.width].copy()
        else:
            img = bg.copy()
        mask = np.zeros((s.height, s.width), bool)
        for o in self.objects:
            px = int(round(_bounce(o["x0"], o["vx"], n, 0.0, s.width - o["w"])))
            py = int(round(_bounce(o["y0"], o["vy"], n, 0.0, s.height - o["h"])))
            sh = o["shape"]
            reg = img[:, py:py + o["h"], px:px + o["w"]]
            reg[:, sh] = o["tex"][:, sh]
            mask[py:py + o["h"], px:px + o["w"]] |= sh
        x = img.reshape(-1) + s.noise * rng.standard_normal(s.m)
        if with_mask:
            return x, mask.reshape(-1)
        return x

    def frames(self, n0, count):
        return np.stack([self.frame(n0 + i) for i in range(count)])


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    video: VideoSpec
    k: int
    mu: float
    n_frames: int
    delta: Optional[float] = None   # None -> derived from mu
    cost: str = "lp"


def small_gray():
    """80x60 grayscale, k=5, 200 frames; rank-3 background with coefficients
    in [0,1]; 3 rectangles over ~5% of the pixels; noise 0.01; mu = 1e-3."""
    v = VideoSpec(80, 60, 1, rank=3, seed=1, noise=0.01, fg_kind="rects",
                  fg_count=3, fg_density=0.05, speed=(1.0, 2.0))
    return Workload("80x60x1 k=5", v, k=5, mu=1e-3, n_frames=200)


def qvga_rgb():
    """320x240 RGB, k=10, 1000 frames; rank-6 background with +-2 px camera
    jitter; ~10% of pixels covered by ellipses moving 1-4 px/frame; noise
    0.02.  delta = 4 * noise, mu = delta^2 (1 - p)."""
    v = VideoSpec(320, 240, 3, rank=6, seed=2, noise=0.02, fg_kind="ellipses",
                  fg_count=6, fg_density=0.10, speed=(1.0, 4.0), jitter=2)
    delta = 0.08
    return Workload("320x240x3 k=10", v, k=10, mu=delta * delta * 0.75, n_frames=1000, delta=delta)


def vga_rgb(stream=0):
    """640x480 RGB, k=15, 1000 frames; the small_gray generator at rank 10."""
    v = VideoSpec(640, 480, 3, rank=10, seed=3, stream=stream, noise=0.01, fg_kind="rects",
                  fg_count=3, fg_density=0.05, speed=(1.0, 2.0))
    return Workload("640x480x3 k=15", v, k=15, mu=1e-3, n_frames=1000)


def mixed_streams(count=64):
    """Independent streams of uneven size: resolution uniform in
    {160x120, 320x240, 640x480} RGB, k uniform in {5, 10, 15} with
    background rank {3, 6, 10}; foreground density uniform in [2%, 20%]
    (3 rectangles); noise 0.01; mu = 1e-3."""
    rng = np.random.default_rng([4, 0xBA7C])
    sizes = [(160, 120), (320, 240), (640, 480)]
    ranks = {5: 3, 10: 6, 15: 10}
    out: List[Workload] = []
    for s in range(count):
        wdt, hgt = sizes[int(rng.integers(0, 3))]
        k = int((5, 10, 15)[int(rng.integers(0, 3))])
        dens = float(rng.uniform(0.02, 0.20))
        v = VideoSpec(wdt, hgt, 3, rank=ranks[k], seed=4, stream=s, noise=0.01, fg_kind="rects",
                      fg_count=3, fg_density=dens, speed=(1.0, 2.0))
        out.append(Workload(f"stream{s} {wdt}x{hgt}x3 k={k}", v, k=k, mu=1e-3, n_frames=1000))
    return out


def lpcost_batch(m=230400, k=10, B=32, seed=5, weighted=False):
    """Differentiable-cost input: U = QR(Gaussian); Y ~ 0.05 N(0, I);
    X = U Y with 10% of entries replaced by U[0,1] outliers, plus N(0, 0.01^2);
    w = 1 (or per-entry weights in {1, 5e-5} when weighted)."""
    rng = np.random.default_rng([seed, 0])
    U = random_orthonormal(m, k, rng)
    Y = 0.05 * rng.standard_normal((k, B))
    X = U @ Y
    out = rng.random((m, B)) < 0.10
    X[out] = rng.uniform(0.0, 1.0, size=int(out.sum()))
    X += 0.01 * rng.standard_normal((m, B))
    if weighted:
        w = np.where(rng.random(m) < 0.1, 5e-5, 1.0)
    else:
        w = np.ones(m)
    return U, Y, X, w


# ---------------------------------------------------------------------------
# Camera-like 8-bit source frames for the ingest path
# ---------------------------------------------------------------------------

class CameraVideo:
    """Interleaved 8-bit frames (H x W x C bytes, as a video decoder writes
    them) at the source resolution: a smooth static scene in [0.2, 0.8],
    `rank` smooth illumination patterns of amplitude 0.06 modulated by
    periodic coefficients, moving rectangles with U[0,1] texture, additive
    N(0, noise^2) (in units of the full range), quantised to 0..255.  The
    ground truth is the set of rectangle pixels.  Frame n is regenerated
    from (seed, n) alone."""

    def __init__(self, width, height, channels=3, rank=3, seed=0, fg_count=3, fg_density=0.05, noise=0.008,
                 speed=(2.0, 6.0)):
        self.width, self.height, self.channels = width, height, channels
        self.seed, self.noise = seed, noise
        rng = np.random.default_rng([seed, 0xCA])
        yy = np.arange(height)[:, None] / height
        xx = np.arange(width)[None, :] / width

        def field():
            f = np.zeros((channels, height, width))
            for c in range(channels):
                for _ in range(3):
                    fy, fx = rng.uniform(0.3, 2.5, size=2)
                    py, px = rng.uniform(0, 2 * math.pi, size=2)
                    f[c] += np.cos(2 * math.pi * fy * yy + py) * np.cos(2 * math.pi * fx * xx + px)
            lo, hi = f.min(), f.max()
            return (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)

        self.base = 0.2 + 0.6 * field()
        self.patterns = [0.06 * (2.0 * field() - 1.0) for _ in range(rank)]
        self.T = rng.uniform(40.0, 160.0, size=rank)
        self.ph = rng.uniform(0.0, 2.0 * math.pi, size=rank)
        self.objects = []
        area = fg_density * width * height / max(fg_count, 1)
        for _ in range(fg_count):
            aspect = rng.uniform(0.6, 1.6)
            bw = min(width, max(1, int(round(math.sqrt(area * aspect)))))
            bh = min(height, max(1, int(round(area / bw))))
            sp = rng.uniform(speed[0], speed[1])
            ang = rng.uniform(0.0, 2.0 * math.pi)
            self.objects.append(dict(w=bw, h=bh, x0=rng.uniform(0, width - bw), y0=rng.uniform(0, height - bh),
                                     vx=sp * math.cos(ang), vy=sp * math.sin(ang),
                                     tex=rng.uniform(0.0, 1.0, size=(channels, bh, bw))))

    def frame(self, n, with_mask=False):
        rng = np.random.default_rng([self.seed, 0xCB, int(n)])
        img = self.base.copy()
        for pat, T, ph in zip(self.patterns, self.T, self.ph):
            img += math.sin(2.0 * math.pi * n / T + ph) * pat
        mask = np.zeros((self.height, self.width), bool)
        for o in self.objects:
            px = int(round(_bounce(o["x0"], o["vx"], n, 0.0, self.width - o["w"])))
            py = int(round(_bounce(o["y0"], o["vy"], n, 0.0, self.height - o["h"])))
            img[:, py:py + o["h"], px:px + o["w"]] = o["tex"]
            mask[py:py + o["h"], px:px + o["w"]] = True
        img += self.noise * rng.standard_normal(img.shape)
        q = np.clip(np.rint(255.0 * img), 0, 255).astype(np.uint8)
        out = np.ascontiguousarray(np.moveaxis(q, 0, 2))
        if with_mask:
            return out, mask.reshape(-1)
        return out
