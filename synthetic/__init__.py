"""Seeded synthetic workloads for the shell fill.

This module only draws inputs: images, label maps (0 = readable, 1 = inpaint,
2 = bystander) and guide fields.  It holds none of the fill's arithmetic and is
shared by the tests, the benchmark and the CPU reference alike.

The paper's own photographs and film are not available, so every workload is
built from the recipes below (the sizes, hole widths and hole fractions follow
the 3D-conversion examples of the paper's numerical section, where the holes are
thin disocclusion "cracks" next to object silhouettes):

* image: per channel a sum of 8 random-phase sinusoids (amplitude U[0,1], phase
  U[0,2pi), direction U[0,2pi), 1..6 cycles per image width), rescaled to
  [0,1], plus random straight step edges (per-channel step U[-0.5,0.5]),
  rescaled to [0,1] again;
* masks: wiggly vertical bands, bands along closed cubic Bezier silhouettes
  (Catmull-Rom tangents) dilated by one pixel, discs, wiggly straight bands;
* guidance: the unit tangent of the nearest of several open cubic splines when
  within 15 px, else the structure-tensor direction tanh((l+ - l-)/Lambda) v-
  of the unmasked image (sigma = 2, rho = 4, Lambda = 1e-5), zero off the hole;
  the same random splines as polylines (segments with unit chord directions)
  are the input of the guide-field construction.

Array conventions: images are H x W x C (row, column, channel); a guide vector
is (gx, gy) with gx along columns and gy along rows.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

__all__ = [
    "Workload",
    "smooth_image",
    "band_mask_c1",
    "silhouette_bands",
    "spline_guidance",
    "spline_segments",
    "degradation_problem",
    "pan_video",
    "pack_segments",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "random_tiny",
    "CONFIG_NAMES",
]


@dataclass
class Workload:
    """One synthetic problem.  `image` is B x H x W x C float32 (or float16),
    `label` B x H x W uint8, `guide` B x H x W x 2 float32."""

    name: str
    image: np.ndarray
    label: np.ndarray
    guide: np.ndarray
    eps: float
    mu: float
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.image.shape

    @property
    def n_hole(self) -> int:
        return int((self.label == 1).sum())


# ----------------------------------------------------------------------------
# images


def smooth_image(rng: np.random.Generator, H: int, W: int, C: int = 3,
                 n_edges: int = 3) -> np.ndarray:
    """Sum of 8 random sinusoids per channel plus `n_edges` step edges, in [0,1]."""
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    img = np.zeros((H, W, C), dtype=np.float64)
    for ch in range(C):
        acc = np.zeros((H, W), dtype=np.float64)
        for _ in range(8):
            amp = rng.uniform(0.0, 1.0)
            phase = rng.uniform(0.0, 2 * math.pi)
            ang = rng.uniform(0.0, 2 * math.pi)
            freq = rng.uniform(1.0, 6.0)
            kx = 2 * math.pi * freq / W * math.cos(ang)
            ky = 2 * math.pi * freq / W * math.sin(ang)
            # sin(a + b) = sin a cos b + cos a sin b, evaluated as outer products
            a = kx * x + phase
            b = ky * y
            acc += amp * (np.sin(a) * np.cos(b) + np.cos(a) * np.sin(b))
        lo, hi = acc.min(), acc.max()
        img[..., ch] = (acc - lo) / max(hi - lo, 1e-12)
    for _ in range(n_edges):
        px, py = rng.uniform(0, W), rng.uniform(0, H)
        ang = rng.uniform(0, 2 * math.pi)
        side = ((x - px) * (-math.sin(ang)) + (y - py) * math.cos(ang)) > 0
        steps = rng.uniform(-0.5, 0.5, size=C)
        img += side[..., None] * steps[None, None, :]
    for ch in range(C):
        lo, hi = img[..., ch].min(), img[..., ch].max()
        img[..., ch] = (img[..., ch] - lo) / max(hi - lo, 1e-12)
    return img.astype(np.float32)


# ----------------------------------------------------------------------------
# curves


def _bezier(p0, p1, p2, p3, t):
    t = t[:, None]
    s = 1.0 - t
    return (s ** 3) * p0 + 3 * (s ** 2) * t * p1 + 3 * s * (t ** 2) * p2 + (t ** 3) * p3


def _bezier_tangent(p0, p1, p2, p3, t):
    t = t[:, None]
    s = 1.0 - t
    return 3 * (s ** 2) * (p1 - p0) + 6 * s * t * (p2 - p1) + 3 * (t ** 2) * (p3 - p2)


def _closed_catmull_rom(knots: np.ndarray, spacing: float = 0.25):
    """Sample a closed composite cubic Bezier through `knots` (K x 2, (x, y))."""
    K = len(knots)
    pts, tans = [], []
    for i in range(K):
        a, b = knots[i], knots[(i + 1) % K]
        prev, nxt = knots[(i - 1) % K], knots[(i + 2) % K]
        c1 = a + (b - prev) / 6.0
        c2 = b - (nxt - a) / 6.0
        length = (np.linalg.norm(c1 - a) + np.linalg.norm(c2 - c1) + np.linalg.norm(b - c2))
        n = max(8, int(math.ceil(length / spacing)))
        t = np.linspace(0.0, 1.0, n, endpoint=False)
        pts.append(_bezier(a, c1, c2, b, t))
        tans.append(_bezier_tangent(a, c1, c2, b, t))
    return np.concatenate(pts), np.concatenate(tans)


def _open_spline(rng, H, W, spacing: float = 0.25):
    """An open cubic Bezier between two random border points."""

    def border_point():
        side = rng.integers(0, 4)
        if side == 0:
            return np.array([rng.uniform(0, W - 1), 0.0])
        if side == 1:
            return np.array([rng.uniform(0, W - 1), H - 1.0])
        if side == 2:
            return np.array([0.0, rng.uniform(0, H - 1)])
        return np.array([W - 1.0, rng.uniform(0, H - 1)])

    p0, p3 = border_point(), border_point()
    p1 = np.array([rng.uniform(0, W - 1), rng.uniform(0, H - 1)])
    p2 = np.array([rng.uniform(0, W - 1), rng.uniform(0, H - 1)])
    length = np.linalg.norm(p1 - p0) + np.linalg.norm(p2 - p1) + np.linalg.norm(p3 - p2)
    n = max(16, int(math.ceil(length / spacing)))
    t = np.linspace(0.0, 1.0, n)
    return _bezier(p0, p1, p2, p3, t), _bezier_tangent(p0, p1, p2, p3, t)


def _raster(points: np.ndarray, H: int, W: int):
    """Nearest-pixel rasterisation; returns (mask, index-of-sample image)."""
    ix = np.rint(points[:, 0]).astype(np.int64)
    iy = np.rint(points[:, 1]).astype(np.int64)
    ok = (ix >= 0) & (ix < W) & (iy >= 0) & (iy < H)
    mask = np.zeros((H, W), dtype=bool)
    idx = np.full((H, W), -1, dtype=np.int64)
    mask[iy[ok], ix[ok]] = True
    idx[iy[ok], ix[ok]] = np.nonzero(ok)[0]
    return mask, idx


# ----------------------------------------------------------------------------
# masks


def band_mask_c1(rng, H: int = 256, W: int = 256, width: int = 8,
                 amp: float = 3.0, period: float = 64.0) -> np.ndarray:
    """Vertical band `width` px wide whose centre wiggles sinusoidally."""
    phi = rng.uniform(0, 2 * math.pi)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    xc = (W - 1) / 2.0 + amp * np.sin(2 * math.pi * y / period + phi)
    return ((x >= xc - width / 2) & (x < xc + width / 2)).astype(np.uint8)


def silhouette_bands(rng, H: int, W: int, n: int = 6, wmin: float = 5.0,
                     wmax: float = 20.0, rmin: float = 60.0, rmax: float = 250.0,
                     target_fraction: float | None = None) -> np.ndarray:
    """Bands of width U[wmin,wmax] along closed Bezier silhouettes, dilated by 1 px.

    With `target_fraction`, silhouettes are added until the hole fraction is
    reached (at least one, at most 64); otherwise exactly `n` are drawn."""
    band = np.zeros((H, W), dtype=bool)
    count = 0
    while True:
        if target_fraction is None and count >= n:
            break
        if target_fraction is not None and (count >= 64 or
                                            (count > 0 and band.mean() >= target_fraction)):
            break
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        rad = rng.uniform(rmin, rmax)
        angles = np.arange(4) * (math.pi / 2) + rng.uniform(0, 2 * math.pi)
        radii = rad * rng.uniform(0.7, 1.3, size=4)
        knots = np.stack([cx + radii * np.cos(angles), cy + radii * np.sin(angles)], axis=1)
        pts, _ = _closed_catmull_rom(knots)
        curve, _ = _raster(pts, H, W)
        if not curve.any():
            continue
        dist = ndimage.distance_transform_edt(~curve)
        w = rng.uniform(wmin, wmax)
        band |= dist <= w / 2.0
        count += 1
    band = ndimage.binary_dilation(band, structure=np.ones((3, 3), dtype=bool))
    return band.astype(np.uint8)


def discs(rng, H: int, W: int, n: int, rmin: float, rmax: float) -> np.ndarray:
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    m = np.zeros((H, W), dtype=bool)
    for _ in range(n):
        cx, cy, r = rng.uniform(0, W), rng.uniform(0, H), rng.uniform(rmin, rmax)
        m |= (x - cx) ** 2 + (y - cy) ** 2 <= r * r
    return m.astype(np.uint8)


def wiggly_bands(rng, H: int, W: int, n: int, wmin: float, wmax: float) -> np.ndarray:
    """Straight bands at random angles with a sinusoidal wiggle of the centre line."""
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    m = np.zeros((H, W), dtype=bool)
    for _ in range(n):
        px, py = rng.uniform(0.2 * W, 0.8 * W), rng.uniform(0.2 * H, 0.8 * H)
        ang = rng.uniform(0, math.pi)
        w = rng.uniform(wmin, wmax)
        amp = rng.uniform(0, 4.0)
        period = rng.uniform(40.0, 160.0)
        t = (x - px) * math.cos(ang) + (y - py) * math.sin(ang)
        d = -(x - px) * math.sin(ang) + (y - py) * math.cos(ang)
        m |= np.abs(d - amp * np.sin(2 * math.pi * t / period)) < w / 2.0
    return m.astype(np.uint8)


# ----------------------------------------------------------------------------
# guidance


def structure_tensor_direction(img: np.ndarray, sigma: float = 2.0, rho: float = 4.0,
                               lam: float = 1e-5) -> np.ndarray:
    """tanh((l+ - l-)/lam) * v- of J_{sigma,rho}, windows (4 sigma + 1)^2, (4 rho + 1)^2."""
    H, W, C = img.shape
    j11 = np.zeros((H, W))
    j12 = np.zeros((H, W))
    j22 = np.zeros((H, W))
    for ch in range(C):
        us = ndimage.gaussian_filter(img[..., ch].astype(np.float64), sigma, truncate=2.0)
        gy, gx = np.gradient(us)
        j11 += gx * gx
        j12 += gx * gy
        j22 += gy * gy
    j11 = ndimage.gaussian_filter(j11, rho, truncate=2.0)
    j12 = ndimage.gaussian_filter(j12, rho, truncate=2.0)
    j22 = ndimage.gaussian_filter(j22, rho, truncate=2.0)
    half_tr = 0.5 * (j11 + j22)
    disc = np.sqrt((0.5 * (j11 - j22)) ** 2 + j12 ** 2)
    lp, lm = half_tr + disc, half_tr - disc
    # eigenvector of the smaller eigenvalue: (j12, lm - j11) or (lm - j22, j12)
    vx1, vy1 = j12, lm - j11
    vx2, vy2 = lm - j22, j12
    use2 = (vx2 ** 2 + vy2 ** 2) > (vx1 ** 2 + vy1 ** 2)
    vx = np.where(use2, vx2, vx1)
    vy = np.where(use2, vy2, vy1)
    nrm = np.sqrt(vx * vx + vy * vy)
    ok = nrm > 0
    vx = np.where(ok, vx / np.where(ok, nrm, 1.0), 0.0)
    vy = np.where(ok, vy / np.where(ok, nrm, 1.0), 0.0)
    mag = np.tanh((lp - lm) / lam)
    return np.stack([mag * vx, mag * vy], axis=-1)


def spline_guidance(rng, img: np.ndarray, label: np.ndarray, n_splines: int = 6,
                    radius: float = 15.0) -> np.ndarray:
    """Unit tangent of the nearest random open spline within `radius` px, else the
    structure-tensor direction; zero off the hole."""
    H, W = label.shape
    pts_all, tan_all = [], []
    for _ in range(n_splines):
        p, t = _open_spline(rng, H, W)
        pts_all.append(p)
        tan_all.append(t)
    pts = np.concatenate(pts_all)
    tans = np.concatenate(tan_all)
    curve, idx = _raster(pts, H, W)
    g = structure_tensor_direction(img)
    if curve.any():
        dist, (iy, ix) = ndimage.distance_transform_edt(~curve, return_indices=True)
        near = idx[iy, ix]
        t = tans[np.clip(near, 0, None)]
        tn = np.linalg.norm(t, axis=-1, keepdims=True)
        t = t / np.where(tn > 0, tn, 1.0)
        close = (dist <= radius)[..., None]
        g = np.where(close, t, g)
    g = np.where((label == 1)[..., None], g, 0.0)
    return g.astype(np.float32)


def spline_segments(rng, H: int, W: int, n_splines: int = 6, spacing: float = 2.0) -> np.ndarray:
    """Random open cubic Beziers between border points (as drawn for
    spline_guidance), each sampled every `spacing` px of control-polygon
    length and returned as a polyline: n x 6 float32 rows (x0, y0, x1, y1, gx,
    gy), (gx, gy) the unit chord direction of the segment."""
    rows = []
    for _ in range(n_splines):
        p, _t = _open_spline(rng, H, W, spacing=spacing)
        d = p[1:] - p[:-1]
        n = np.linalg.norm(d, axis=1)
        keep = n > 0
        d = d[keep] / n[keep, None]
        rows.append(np.concatenate([p[:-1][keep], p[1:][keep], d], axis=1))
    if not rows:
        return np.zeros((0, 6), dtype=np.float32)
    return np.concatenate(rows).astype(np.float32)


def pack_segments(frames) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate per-frame segment arrays into (seg n x 6 float32, seg_off
    int32[B + 1])."""
    frames = [np.asarray(f, dtype=np.float32).reshape(-1, 6) for f in frames]
    off = np.zeros(len(frames) + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(f) for f in frames])
    seg = np.concatenate(frames) if frames else np.zeros((0, 6), dtype=np.float32)
    return np.ascontiguousarray(seg, dtype=np.float32), off


@dataclass
class DegradationProblem:
    """The signal-degradation study of Sec. 4: the band |y - tan(a) x| <= 0.1
    on Omega = [-1, 1] x [-0.5, 0.5] with the hole D = (-0.8, 0.8) x
    (-0.3, 0.3), rendered at W x W/2 pixels (h = 2 / W, pixel centres), the
    guide along the band.  `exact` is the continuum solution sampled at the
    pixel centres (the band carried straight across D); x, y the centres."""

    image: np.ndarray   # H x W x 1 float32, 0 on the hole
    label: np.ndarray   # H x W uint8
    guide: np.ndarray   # H x W x 2 float32, (cos a, -sin a) on the hole
    exact: np.ndarray   # H x W float64
    x: np.ndarray       # W pixel-centre abscissae
    y: np.ndarray       # H pixel-centre ordinates (row 0 at the top)
    h: float


def degradation_problem(W: int, angle_deg: float = 73.0, half_width: float = 0.1):
    H = W // 2
    h = 2.0 / W
    x = -1.0 + (np.arange(W) + 0.5) * h
    y = 0.5 - (np.arange(H) + 0.5) * h
    X, Y = np.meshgrid(x, y)
    t = math.tan(math.radians(angle_deg))
    exact = (np.abs(Y - t * X) <= half_width).astype(np.float64)
    hole = (np.abs(X) < 0.8) & (np.abs(Y) < 0.3)
    img = np.where(hole, 0.0, exact)[..., None].astype(np.float32)
    g = np.zeros((H, W, 2), dtype=np.float32)
    g[..., 0] = np.float32(math.cos(math.radians(angle_deg)))
    g[..., 1] = np.float32(-math.sin(math.radians(angle_deg)))  # rows grow downwards
    g[~hole] = 0.0
    return DegradationProblem(img, hole.astype(np.uint8), g, exact, x, y, h)


def pan_video(seed: int = 6, B: int = 16, H: int = 1080, W: int = 1920, step=(3, 1),
              margin: int = 8, dtype=np.float16):
    """A camera pan over one static scene: frame t is the H x W window of a
    larger canvas moved by t * step = (dx, dy) pixels; the canvas carries six
    silhouette bands (the disocclusion holes of the full-HD recipe) and the
    spline / structure-tensor guide.  Holes are kept at least `margin` pixels
    from every frame border.  Returns (Workload of B frames, per-frame (x0, y0)
    window origins in the canvas)."""
    rng = np.random.default_rng(seed)
    dx, dy = step
    CW, CH = W + dx * (B - 1), H + dy * (B - 1)
    img, label, guide = _frame_c2(rng, CH, CW)
    origins = [(t * dx, t * dy) for t in range(B)]
    # holes only where every frame sees them at least `margin` px inside
    keep = np.zeros((CH, CW), dtype=bool)
    keep[dy * (B - 1) + margin:H - margin, dx * (B - 1) + margin:W - margin] = True
    label = np.where((label == 1) & ~keep, np.uint8(0), label)
    guide = np.where((label == 1)[..., None], guide, np.float32(0)).astype(np.float32)
    frames = [(img[y0:y0 + H, x0:x0 + W], label[y0:y0 + H, x0:x0 + W],
               guide[y0:y0 + H, x0:x0 + W]) for x0, y0 in origins]
    wl = Workload("pan", np.stack([f[0] for f in frames]).astype(dtype),
                  np.stack([f[1] for f in frames]), np.stack([f[2] for f in frames]), 3.0, 50.0,
                  {"seed": seed, "B": B, "H": H, "W": W, "step": list(step)})
    return wl, origins


def constant_guidance(H: int, W: int, angle_deg: float, label: np.ndarray) -> np.ndarray:
    a = math.radians(angle_deg)
    g = np.zeros((H, W, 2), dtype=np.float32)
    g[..., 0] = np.float32(math.cos(a))
    g[..., 1] = np.float32(math.sin(a))
    return np.where((label == 1)[..., None], g, np.float32(0)).astype(np.float32)


def smooth_angle_field(rng, H: int, W: int, n: int = 4) -> np.ndarray:
    """Smooth random angle field in [0, pi): 4 sinusoids at 0.5..2 cycles/image."""
    y = np.arange(H, dtype=np.float64)[:, None] / H
    x = np.arange(W, dtype=np.float64)[None, :] / W
    f = np.zeros((H, W))
    for _ in range(n):
        fx, fy = rng.uniform(0.5, 2.0, size=2) * rng.choice([-1, 1], size=2)
        f += rng.uniform(0.5, 1.0) * np.sin(2 * math.pi * (fx * x + fy * y) + rng.uniform(0, 2 * math.pi))
    lo, hi = f.min(), f.max()
    return (math.pi * (f - lo) / max(hi - lo, 1e-12) * (1 - 1e-6)).astype(np.float32)


# ----------------------------------------------------------------------------
# the five configurations


CONFIG_NAMES = {
    1: "plain 256x256 RGB fp32, wiggly 8-px band, constant 30 deg guide, eps=3, mu=50",
    2: "plain 1920x1080 RGB fp32, 6 silhouette bands 5-20 px, spline/structure-tensor guide, eps=3, mu=50",
    3: "plain 3840x2160 RGB fp32, 200-px wiggly band + 20 discs, eps=5, mu=100",
    4: "batched 64x1920x1080 RGB fp16 storage, lognormal hole fraction, eps=3, mu=50",
    5: "differentiable 16x512x512 RGB fp32, band masks 6-16 px, smooth angle field, eps=3, mu=50",
}


def config1(seed: int = 1, H: int = 256, W: int = 256) -> Workload:
    rng = np.random.default_rng(seed)
    img = smooth_image(rng, H, W, 3, n_edges=3)
    label = band_mask_c1(rng, H, W)
    guide = constant_guidance(H, W, 30.0, label)
    return Workload("c1", img[None], label[None], guide[None], 3.0, 50.0,
                    {"seed": seed, "H": H, "W": W})


def _frame_c2(rng, H, W, n_sil=6, target_fraction=None):
    img = smooth_image(rng, H, W, 3, n_edges=12)
    label = silhouette_bands(rng, H, W, n=n_sil, target_fraction=target_fraction)
    guide = spline_guidance(rng, img, label)
    return img, label, guide


def config2(seed: int = 2, H: int = 1080, W: int = 1920) -> Workload:
    rng = np.random.default_rng(seed)
    img, label, guide = _frame_c2(rng, H, W)
    return Workload("c2", img[None], label[None], guide[None], 3.0, 50.0,
                    {"seed": seed, "H": H, "W": W})


def config3(seed: int = 3, H: int = 2160, W: int = 3840) -> Workload:
    rng = np.random.default_rng(seed)
    img = smooth_image(rng, H, W, 3, n_edges=12)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    xc = W / 2.0 + 20.0 * np.sin(2 * math.pi * y / 400.0)
    band = (np.abs(x - xc) < 100.0 * W / 3840.0)
    label = (band | discs(rng, H, W, 20, 10.0, 60.0).astype(bool)).astype(np.uint8)
    guide = spline_guidance(rng, img, label)
    return Workload("c3", img[None], label[None], guide[None], 5.0, 100.0,
                    {"seed": seed, "H": H, "W": W})


def _frame_c4(args):
    seed, f, H, W = args
    rng = np.random.default_rng([seed, f])
    frac = float(np.clip(rng.lognormal(math.log(0.02), 0.5), 0.005, 0.08))
    img, label, guide = _frame_c2(rng, H, W, target_fraction=frac)
    return img.astype(np.float16), label, guide, frac


def _map_frames(fn, jobs, workers):
    if workers is None:
        workers = min(len(jobs), os.cpu_count() or 1, 16)
    if workers <= 1 or len(jobs) <= 1:
        return [fn(j) for j in jobs]
    # threads, not processes: the array work releases the GIL, and nothing is
    # forked from a process that may already drive a GPU
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(workers) as pool:
        return list(pool.map(fn, jobs))


def config4(seed: int = 4, B: int = 64, H: int = 1080, W: int = 1920,
            workers: int | None = None) -> Workload:
    """Frame f is drawn from rng([seed, f]) alone, so any subset of frames
    can be regenerated independently (frames=...)."""
    res = _map_frames(_frame_c4, [(seed, f, H, W) for f in range(B)], workers)
    return Workload("c4", np.stack([r[0] for r in res]), np.stack([r[1] for r in res]),
                    np.stack([r[2] for r in res]), 3.0, 50.0,
                    {"seed": seed, "B": B, "H": H, "W": W,
                     "target_fractions": [r[3] for r in res]})


def config5(seed: int = 5, B: int = 16, H: int = 512, W: int = 512):
    """Returns (Workload, theta) where theta is the B x H x W angle field; the
    workload's guide is (cos theta, sin theta) on the hole, zero elsewhere."""
    imgs, labels, thetas = [], [], []
    for f in range(B):
        rng = np.random.default_rng([seed, f])
        imgs.append(smooth_image(rng, H, W, 3, n_edges=12))
        labels.append(wiggly_bands(rng, H, W, 3, 6.0, 16.0))
        thetas.append(smooth_angle_field(rng, H, W))
    label = np.stack(labels)
    theta = np.stack(thetas)
    g = np.stack([np.cos(theta), np.sin(theta)], axis=-1).astype(np.float32)
    g = np.where((label == 1)[..., None], g, np.float32(0)).astype(np.float32)
    return (Workload("c5", np.stack(imgs), label, g, 3.0, 50.0,
                     {"seed": seed, "B": B, "H": H, "W": W}), theta)


def random_tiny(rng, H: int, W: int, C: int = 2, p_hole: float = 0.35,
                p_bystander: float = 0.1, blob: bool = True, zero_guide_frac: float = 0.1):
    """Small random problem with holes (often touching the image border),
    bystanders and random guidance (some zero vectors, random magnitudes)."""
    img = rng.uniform(0, 1, size=(H, W, C)).astype(np.float32)
    if blob:
        noise = ndimage.gaussian_filter(rng.normal(size=(H, W)), 1.5)
        thr = np.quantile(noise, 1 - p_hole)
        hole = noise >= thr
    else:
        hole = rng.uniform(size=(H, W)) < p_hole
    label = hole.astype(np.uint8)
    bys = (rng.uniform(size=(H, W)) < p_bystander) & ~hole
    label[bys] = 2
    ang = rng.uniform(0, 2 * math.pi, size=(H, W))
    mag = rng.uniform(0.05, 1.0, size=(H, W))
    mag[rng.uniform(size=(H, W)) < zero_guide_frac] = 0.0
    g = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=-1).astype(np.float32)
    g = np.where((label == 1)[..., None], g, np.float32(0)).astype(np.float32)
    return img, label, g
