"""Seeded synthetic ring images: the shared input generator.

This module draws frames of fluorescent-particle ring patterns with known ground truth.
It holds none of the detection method's arithmetic: it only renders an intensity model
and adds noise.  Both the GPU path and the CPU oracle are fed from here; nothing else is
shared between them.

Ring model (point-sampled at integer pixel centres, x = column, y = row):

    I(p) = bg(p) + sum_j A_j * exp(-(|p - c_j| - R_j)^2 / (2 s_j^2))

Each ring is rendered inside its bounding box widened by 6 s_j; the truncated tail is
below 2e-8 of the amplitude.

The workload recipes follow the problem statement of the paper (Results, "Problem
statement": an image of rings whose centres and radii are wanted) with the sizes and
distributions given in each recipe's docstring.  The paper's own images are not available,
so these synthetic frames stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------------------
# default detection parameters per workload (plain numbers: the curvature threshold sits at
# a quarter of the weakest ring's smoothed curvature)
# ----------------------------------------------------------------------------------------
PARAMS_C1 = dict(sigma_smooth=2.0, k_threshold=-0.02, r_min=8, r_max=40, vote_threshold=3,
                 peak_fraction=0.4, sig_slope=0.05, sig_icpt=0.25, annulus_halfwidth=2,
                 min_fit_points=8)
PARAMS_C2 = dict(PARAMS_C1, k_threshold=-7.0, r_min=5, r_max=70)
PARAMS_C3 = dict(PARAMS_C1, k_threshold=-20.0, r_min=8, r_max=40)
PARAMS_C4 = dict(PARAMS_C1, k_threshold=-0.015, r_min=8, r_max=40)
PARAMS_C5 = dict(PARAMS_C1, k_threshold=-20.0, r_min=8, r_max=80)

BATCH_SIZES = ((512, 512), (1024, 768), (1280, 1024), (2048, 1088))  # (width, height)


@dataclasses.dataclass
class Frame:
    """One synthetic frame plus its ground truth."""
    image: np.ndarray          # (H, W) uint16 or float32
    cx: np.ndarray             # (n,) float64, column of each ring centre
    cy: np.ndarray             # (n,) float64, row of each ring centre
    R: np.ndarray              # (n,) float64, ring radius
    s: np.ndarray              # (n,) float64, radial profile sigma
    A: np.ndarray              # (n,) float64, amplitude (image units)
    params: dict               # default detection parameters for this workload
    seed: int = 0

    @property
    def height(self) -> int:
        return self.image.shape[0]

    @property
    def width(self) -> int:
        return self.image.shape[1]


def render(W: int, H: int, bg: np.ndarray, cx, cy, R, s, A) -> np.ndarray:
    """Clean float64 intensity: background plus Gaussian-profile rings."""
    img = np.array(bg, dtype=np.float64, copy=True)
    if img.shape != (H, W):
        img = np.broadcast_to(img, (H, W)).copy()
    for j in range(len(R)):
        ext = R[j] + 6.0 * s[j]
        x0 = max(0, int(math.floor(cx[j] - ext)))
        x1 = min(W - 1, int(math.ceil(cx[j] + ext)))
        y0 = max(0, int(math.floor(cy[j] - ext)))
        y1 = min(H - 1, int(math.ceil(cy[j] + ext)))
        if x1 < x0 or y1 < y0:
            continue
        xs = np.arange(x0, x1 + 1, dtype=np.float64)
        ys = np.arange(y0, y1 + 1, dtype=np.float64)
        rho = np.hypot(xs[None, :] - cx[j], ys[:, None] - cy[j])
        img[y0:y1 + 1, x0:x1 + 1] += A[j] * np.exp(-((rho - R[j]) ** 2) / (2.0 * s[j] ** 2))
    return img


def _lens_fraction(d, r1, r2):
    """Area of the intersection of two discs divided by the smaller disc's area."""
    d = np.asarray(d, dtype=np.float64)
    r1 = np.broadcast_to(np.asarray(r1, np.float64), d.shape)
    r2 = np.broadcast_to(np.asarray(r2, np.float64), d.shape)
    small = np.minimum(r1, r2)
    out = np.zeros_like(d)
    inside = d <= np.abs(r1 - r2)
    out[inside] = 1.0
    part = (~inside) & (d < r1 + r2)
    if np.any(part):
        dd, a, b = d[part], r1[part], r2[part]
        c1 = np.clip((dd * dd + a * a - b * b) / (2 * dd * a), -1.0, 1.0)
        c2 = np.clip((dd * dd + b * b - a * a) / (2 * dd * b), -1.0, 1.0)
        area = (a * a * np.arccos(c1) + b * b * np.arccos(c2)
                - 0.5 * np.sqrt(np.maximum((-dd + a + b) * (dd + a - b) * (dd - a + b) * (dd + a + b), 0.0)))
        out[part] = area / (np.pi * small[part] ** 2)
    return out


def place_rings(rng: np.random.Generator, W: int, H: int, n: int, draw_radius, *,
                margin: float | None = None, max_overlap: float | None = None,
                max_attempts: int = 300_000, batch: int = 2048):
    """Rejection-sample ring centres uniform in [0, W-1] x [0, H-1].

    Exactly one of ``margin`` (discs disjoint with that gap) or ``max_overlap`` (lens area
    over the smaller disc's area at most this fraction) constrains the placement.
    Candidates are proposed in batches; the accepted set is the same as proposing them one
    at a time in the same order.
    """
    cx = np.empty(0)
    cy = np.empty(0)
    R = np.empty(0)
    attempts = 0
    while len(R) < n and attempts < max_attempts:
        m = min(batch, max_attempts - attempts)
        px = rng.uniform(0.0, W - 1.0, m)
        py = rng.uniform(0.0, H - 1.0, m)
        pr = draw_radius(rng, m)
        attempts += m
        # conflicts with rings placed before this batch
        if len(R):
            d = np.hypot(px[:, None] - cx[None, :], py[:, None] - cy[None, :])
            if margin is not None:
                bad = np.any(d < pr[:, None] + R[None, :] + margin, axis=1)
            else:
                bad = np.any(_lens_fraction(d, pr[:, None], R[None, :]) > max_overlap, axis=1)
        else:
            bad = np.zeros(m, dtype=bool)
        acc_x, acc_y, acc_r = [], [], []
        for i in range(m):
            if len(R) + len(acc_r) >= n:
                break
            if bad[i]:
                continue
            if acc_r:
                ax = np.asarray(acc_x)
                ay = np.asarray(acc_y)
                ar = np.asarray(acc_r)
                d = np.hypot(px[i] - ax, py[i] - ay)
                if margin is not None:
                    if np.any(d < pr[i] + ar + margin):
                        continue
                elif np.any(_lens_fraction(d, pr[i], ar) > max_overlap):
                    continue
            acc_x.append(px[i])
            acc_y.append(py[i])
            acc_r.append(pr[i])
        if acc_r:
            cx = np.concatenate([cx, acc_x])
            cy = np.concatenate([cy, acc_y])
            R = np.concatenate([R, acc_r])
    return cx, cy, R


def _uniform(lo, hi):
    return lambda rng, m: rng.uniform(lo, hi, m)


def config1(seed: int = 0) -> Frame:
    """256x256 float32: background 0.2, 8 disjoint rings, R ~ U(10, 30), s = 1.5, A = 1,
    additive N(0, 0.05^2) noise."""
    W = H = 256
    rng = np.random.Generator(np.random.PCG64(seed))
    s0 = 1.5
    cx, cy, R = place_rings(rng, W, H, 8, _uniform(10.0, 30.0), margin=3 * s0)
    n = len(R)
    s = np.full(n, s0)
    A = np.ones(n)
    img = render(W, H, np.full((H, W), 0.2), cx, cy, R, s, A)
    img = img + rng.normal(0.0, 0.05, img.shape)
    return Frame(img.astype(np.float32), cx, cy, R, s, A, dict(PARAMS_C1), seed)


def _counts(rng, clean, read_sigma):
    """Poisson shot noise plus Gaussian read noise, rounded and clipped to 12 bits."""
    shot = rng.poisson(np.maximum(clean, 0.0)).astype(np.float64)
    val = np.rint(shot + rng.normal(0.0, read_sigma, clean.shape))
    return np.clip(val, 0, 4095).astype(np.uint16)


def config2(seed: int = 1, W: int = 1024, H: int = 1024, n_rings: int = 200) -> Frame:
    """1024x1024 uint16, 12-bit: background ramp 300 -> 600 counts along x, 200 rings with
    R ~ U(8, 60), s ~ U(1, 2.5), A ~ U(400, 1200) counts, pairwise overlap (lens area over
    the smaller disc) at most 30 %, Poisson shot noise plus N(0, 10^2) read noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cx, cy, R = place_rings(rng, W, H, n_rings, _uniform(8.0, 60.0), max_overlap=0.30)
    n = len(R)
    s = rng.uniform(1.0, 2.5, n)
    A = rng.uniform(400.0, 1200.0, n)
    bg = 300.0 + 300.0 * np.arange(W, dtype=np.float64)[None, :] / (W - 1)
    clean = render(W, H, np.broadcast_to(bg, (H, W)), cx, cy, R, s, A)
    img = _counts(rng, clean, 10.0)
    return Frame(img, cx, cy, R, s, A, dict(PARAMS_C2), seed)


def _c1_geometry_counts(rng, W, H, n_rings, r_lo=10.0, r_hi=30.0, max_attempts=300_000):
    s0 = 1.5
    cx, cy, R = place_rings(rng, W, H, n_rings, _uniform(r_lo, r_hi), margin=3 * s0,
                            max_attempts=max_attempts)
    n = len(R)
    s = np.full(n, s0)
    A = np.full(n, 1000.0)
    clean = render(W, H, np.full((H, W), 200.0), cx, cy, R, s, A)
    val = np.rint(clean + rng.normal(0.0, 50.0, clean.shape))
    img = np.clip(val, 0, 4095).astype(np.uint16)
    return img, cx, cy, R, s, A


def config3_plan(seed: int = 2, n_frames: int = 64) -> list[tuple]:
    """(width, height, rings asked for, frame seed) of each frame of the uneven batch."""
    ss = np.random.SeedSequence(seed)
    top = np.random.Generator(np.random.PCG64(ss))
    children = ss.spawn(n_frames)
    plan = []
    for i in range(n_frames):
        W, H = BATCH_SIZES[int(top.integers(0, len(BATCH_SIZES)))]
        n_rings = int(top.integers(50, 801))
        plan.append((W, H, n_rings, children[i]))
    return plan


def config3_frame(item, seed: int = 2, max_attempts: int = 300_000) -> Frame:
    """One frame of the uneven batch from its plan entry (frames can be made in parallel)."""
    W, H, n_rings, child = item
    rng = np.random.Generator(np.random.PCG64(child))
    img, cx, cy, R, s, A = _c1_geometry_counts(rng, W, H, n_rings, max_attempts=max_attempts)
    return Frame(img, cx, cy, R, s, A, dict(PARAMS_C3), seed)


def config3(seed: int = 2, n_frames: int = 64, max_attempts: int = 300_000) -> list[Frame]:
    """Batch of uint16 frames of uneven sizes from BATCH_SIZES, 50..800 disjoint rings each
    with the 256x256 geometry (R ~ U(10, 30), s = 1.5), intensities x1000 counts
    (background 200, amplitude 1000, Gaussian noise sigma 50), 12-bit."""
    return [config3_frame(item, seed, max_attempts) for item in config3_plan(seed, n_frames)]


def config2_batch(seed0: int = 1000, n_frames: int = 64, W: int = 1024, H: int = 1024) -> list[Frame]:
    """Many 1024x1024 frames drawn like config2 with seeds seed0, seed0+1, ..."""
    return [config2(seed0 + i, W, H) for i in range(n_frames)]


def config4(seed: int = 3, n_frames: int = 16, W: int = 1024, H: int = 1024,
            n_rings: int = 300) -> list[Frame]:
    """float32 frames with the 256x256 ring distributions, min-max normalised to [0, 1]."""
    ss = np.random.SeedSequence(seed)
    frames = []
    for child in ss.spawn(n_frames):
        rng = np.random.Generator(np.random.PCG64(child))
        s0 = 1.5
        cx, cy, R = place_rings(rng, W, H, n_rings, _uniform(10.0, 30.0), margin=3 * s0)
        n = len(R)
        s = np.full(n, s0)
        A = np.ones(n)
        img = render(W, H, np.full((H, W), 0.2), cx, cy, R, s, A)
        img = img + rng.normal(0.0, 0.05, img.shape)
        lo, hi = img.min(), img.max()
        scale = 1.0 / (hi - lo)
        img = (img - lo) * scale
        frames.append(Frame(img.astype(np.float32), cx, cy, R, s, A * scale,
                            dict(PARAMS_C4), seed))
    return frames


class Stream:
    """2048x2048 uint16 sequence: 1000 rings on reflecting Gaussian random walks (sigma 1.5 px
    per frame in x and y), depth z in [0, 1] on a reflecting walk (sigma 0.01 per frame) and
    radius(z) = 8 + 72 z^2; background, noise and amplitude as the x1000-count batch frames.
    Frame t is reproducible from (seed, t) alone, so a run can resume at any frame."""

    def __init__(self, seed: int = 4, W: int = 2048, H: int = 2048, n_rings: int = 1000):
        self.seed, self.W, self.H, self.n = seed, W, H, n_rings
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0])))
        self.x0 = rng.uniform(0, W - 1, n_rings)
        self.y0 = rng.uniform(0, H - 1, n_rings)
        self.z0 = rng.uniform(0, 1, n_rings)

    @staticmethod
    def _reflect(v, lo, hi):
        span = hi - lo
        v = np.mod(v - lo, 2 * span)
        return lo + np.where(v > span, 2 * span - v, v)

    def state(self, t: int):
        """Ring positions and depth at frame t (walk increments drawn per frame)."""
        x, y, z = self.x0.copy(), self.y0.copy(), self.z0.copy()
        for k in range(1, t + 1):
            rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed, 1, k])))
            x = self._reflect(x + rng.normal(0, 1.5, self.n), 0.0, self.W - 1.0)
            y = self._reflect(y + rng.normal(0, 1.5, self.n), 0.0, self.H - 1.0)
            z = self._reflect(z + rng.normal(0, 0.01, self.n), 0.0, 1.0)
        return x, y, z

    def trajectories(self, n_frames: int):
        """Positions and depths of every ring at frames 0 .. n_frames - 1, arrays (n_frames, n):
        the walk of state(t) drawn once, with the same increments."""
        xs = np.empty((n_frames, self.n))
        ys = np.empty((n_frames, self.n))
        zs = np.empty((n_frames, self.n))
        x, y, z = self.x0.copy(), self.y0.copy(), self.z0.copy()
        for k in range(n_frames):
            if k > 0:
                rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed, 1, k])))
                x = self._reflect(x + rng.normal(0, 1.5, self.n), 0.0, self.W - 1.0)
                y = self._reflect(y + rng.normal(0, 1.5, self.n), 0.0, self.H - 1.0)
                z = self._reflect(z + rng.normal(0, 0.01, self.n), 0.0, 1.0)
            xs[k], ys[k], zs[k] = x, y, z
        return xs, ys, zs

    @staticmethod
    def radius(z):
        """radius(z) = 8 + 72 z^2."""
        return 8.0 + 72.0 * np.asarray(z) ** 2

    def render_device(self, x, y, z, out, generator):
        """The frame of ring state (x, y, z) rendered by torch on out's device into out (int16
        [H, W], values 0 .. 4095, bit-identical to uint16): background 200, amplitude 1000,
        profile sigma 1.5, N(0, 50^2) noise from `generator`, rounded and clipped to 12 bits.
        Same model as frame(t), evaluated in float32 with the device's noise stream, so the
        pixels are not numpy's; used where thousands of frames are needed quickly."""
        import torch
        img = render_torch(self.W, self.H, 200.0, x, y, self.radius(z), np.full(self.n, 1.5),
                           np.full(self.n, 1000.0), out.device)
        img += torch.randn(img.shape, device=out.device, generator=generator) * 50.0
        out.copy_(torch.clamp(torch.round(img), 0.0, 4095.0).to(torch.int16))
        return out

    def frame(self, t: int) -> Frame:
        x, y, z = self.state(t)
        R = 8.0 + 72.0 * z * z
        s = np.full(self.n, 1.5)
        A = np.full(self.n, 1000.0)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed, 2, t])))
        clean = render(self.W, self.H, np.full((self.H, self.W), 200.0), x, y, R, s, A)
        img = np.clip(np.rint(clean + rng.normal(0.0, 50.0, clean.shape)), 0, 4095).astype(np.uint16)
        return Frame(img, x, y, R, s, A, dict(PARAMS_C5), self.seed)


def render_torch(W: int, H: int, bg: float, cx, cy, R, s, A, device, bucket: int = 16):
    """render() with torch on `device` in float32 (constant background): each ring is evaluated
    on its box [floor(c - ext), ceil(c + ext)] (ext = R + 6 s) clipped to the frame, the rings
    grouped by box size in steps of `bucket` px, and added with index_add_.  Agrees with
    render() to float32 rounding."""
    import torch
    cx, cy, R, s, A = (np.asarray(v, dtype=np.float64) for v in (cx, cy, R, s, A))
    img = torch.full((H * W,), float(bg), dtype=torch.float32, device=device)
    ext = R + 6.0 * s
    lo_x, hi_x = np.floor(cx - ext), np.ceil(cx + ext)
    lo_y, hi_y = np.floor(cy - ext), np.ceil(cy + ext)
    side = np.maximum(hi_x - lo_x, hi_y - lo_y).astype(np.int64) + 1
    group = (side + bucket - 1) // bucket
    for g in np.unique(group):
        sel = np.nonzero(group == g)[0]
        B = int(g) * bucket
        t = lambda v: torch.as_tensor(v[sel], dtype=torch.float32, device=device)[:, None, None]
        x0, y0 = t(lo_x), t(lo_y)
        off = torch.arange(B, dtype=torch.float32, device=device)
        X = x0 + off[None, None, :]
        Y = y0 + off[None, :, None]
        ok = (X <= t(hi_x)) & (Y <= t(hi_y)) & (X >= 0) & (X <= W - 1) & (Y >= 0) & (Y <= H - 1)
        rho = torch.hypot(X - t(cx), Y - t(cy))
        val = t(A) * torch.exp(-((rho - t(R)) ** 2) / (2.0 * t(s) ** 2))
        idx = (Y * W + X).to(torch.int64)
        img.index_add_(0, idx[ok], val[ok])
    return img.view(H, W)


def single_ring(W: int, H: int, cx: float, cy: float, R: float, s: float = 1.5, A: float = 1.0,
                bg: float = 0.0) -> Frame:
    """One noise-free ring, float32."""
    img = render(W, H, np.full((H, W), bg), np.array([cx]), np.array([cy]), np.array([R]),
                 np.array([s]), np.array([A]))
    p = dict(PARAMS_C1)
    return Frame(img.astype(np.float32), np.array([cx]), np.array([cy]), np.array([R]),
                 np.array([s]), np.array([A]), p, 0)
