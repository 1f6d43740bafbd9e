"""Seeded synthetic inputs for object-removal workloads.

This module only draws images and masks.  It holds none of the removal
method's arithmetic, so both the HIP path and the CPU oracle can consume its
output.  All randomness comes from ``numpy.random.default_rng`` with sub-seeds
from ``SeedSequence(seed).spawn``; only +, -, *, / and integer operations are
used (no transcendental functions), so the bytes are identical on any IEEE
machine with the same numpy.

The paper evaluates on four natural photographs with masks drawn by hand
(WalkingMan 512x384, River 480x639, DivingMan 576x384, Hill 1024x550); those
are not available, and these generators stand in for them with textured,
edged and noisy content plus blob-shaped holes of the stated sizes.

Workloads:
  small    128x96, smooth gradients + 8 textured rectangles + noise,
           elliptical 24x20 hole, 9x9 patch, full search.
  vga      640x480 value-noise texture mix + 10 straight edges, one irregular
           blob hole of about 8% of the area, 9x9 patch, full search.
  hd       1920x1080, 12 Voronoi regions of periodic textures + gradient +
           noise, one blob hole of about 5%; 9x9 / 13x13 patch, full search or
           the alpha = 1 window (3x the hole's bounding box).
  batch    64 images of uneven size 320x240 .. 1280x720, 1-3 blobs covering
           2-10%, 9x9 patch.
  serving  Poisson arrivals of jobs 256x256 .. 2048x1536, 1-10% holes with
           1-3 blobs, patch 7/9/11.
  paper    stand-ins shaped like the paper's four photographs (Table 3):
           WalkingMan 512x384 with a 78x126 object, River 480x639 with a
           59x93 object, DivingMan 576x384 with a 155x186 object, Hill
           1024x550 with a 1024x10 strip; value-noise + edge content.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

SEARCH_FULL, SEARCH_ALPHA, SEARCH_RECT = 0, 1, 2


@dataclasses.dataclass
class Job:
    """One removal job: image, hole mask and parameters."""
    name: str
    rgb: np.ndarray          # uint8 [H, W, 3]
    mask: np.ndarray         # uint8 [H, W], 1 = pixel to remove
    patch_radius: int = 4
    search_mode: int = SEARCH_FULL
    alpha: tuple = (0, 1)    # search factor as a rational (num, den)
    rect: tuple = (0, 0, 0, 0)
    arrival_s: float = 0.0   # serving only

    @property
    def width(self) -> int:
        return int(self.rgb.shape[1])

    @property
    def height(self) -> int:
        return int(self.rgb.shape[0])

    def sha256(self) -> str:
        return input_sha256(self.rgb, self.mask)


def input_sha256(rgb: np.ndarray, mask: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(rgb.shape, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(rgb, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(mask, dtype=np.uint8).tobytes())
    return h.hexdigest()


def _rngs(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def _to_u8(v: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


# ------------------------------------------------------------------ content

def content_gradient_rects(W: int, H: int, rng: np.random.Generator, n_rects: int = 8) -> np.ndarray:
    """Smooth per-channel gradients plus textured rectangles plus noise."""
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.empty((H, W, 3), dtype=np.float64)
    for c in range(3):
        base = rng.uniform(40, 200)
        sx, sy = rng.uniform(-0.6, 0.6, size=2)
        img[..., c] = base + sx * (x - W / 2) + sy * (y - H / 2)
    for _ in range(n_rects):
        w, h = rng.integers(8, 41, size=2)
        x0 = int(rng.integers(0, max(W - w, 1)))
        y0 = int(rng.integers(0, max(H - h, 1)))
        kind = int(rng.integers(0, 5))
        contrast = rng.uniform(30, 60)
        color = rng.uniform(30, 220, size=3)
        yy, xx = np.mgrid[0:h, 0:w]
        if kind == 0:                      # checker
            cell = int(rng.integers(2, 7))
            pat = ((xx // cell + yy // cell) % 2).astype(np.float64)
        elif kind == 1:                    # horizontal stripes
            per = int(rng.integers(3, 9))
            pat = ((yy % per) < per // 2).astype(np.float64)
        elif kind == 2:                    # vertical stripes
            per = int(rng.integers(3, 9))
            pat = ((xx % per) < per // 2).astype(np.float64)
        elif kind == 3:                    # diagonal stripes
            per = int(rng.integers(3, 9))
            pat = (((xx + yy) % per) < per // 2).astype(np.float64)
        else:                              # random dots
            pat = (rng.random((h, w)) < 0.3).astype(np.float64)
        img[y0:y0 + h, x0:x0 + w, :] = color[None, None, :] + contrast * pat[..., None]
    img += rng.integers(-8, 9, size=(H, W, 3))
    return _to_u8(img)


def _value_noise(W: int, H: int, spacing: int, rng: np.random.Generator) -> np.ndarray:
    """Lattice value noise with smoothstep interpolation, values in [-1, 1].

    Interpolates along x once per lattice row, then between lattice rows;
    every pixel sees the same arithmetic as a direct per-pixel evaluation.
    """
    gw, gh = W // spacing + 2, H // spacing + 2
    lat = rng.uniform(-1.0, 1.0, size=(gh, gw))
    x = np.arange(W)
    y = np.arange(H)
    fx = (x % spacing).astype(np.float64) / spacing
    fy = (y % spacing).astype(np.float64) / spacing
    ix, iy = x // spacing, y // spacing
    sx = fx * fx * (3.0 - 2.0 * fx)
    sy = fy * fy * (3.0 - 2.0 * fy)
    a, b = lat[:, ix], lat[:, ix + 1]          # [gh, W]
    rows = a + (b - a) * sx[None, :]           # x-interpolated lattice rows
    top, bot = rows[iy], rows[iy + 1]          # [H, W]
    return top + (bot - top) * sy[:, None]


def content_noise_edges(W: int, H: int, rng: np.random.Generator, n_edges: int = 10) -> np.ndarray:
    """Five-octave value-noise mix plus straight half-plane edges."""
    img = np.full((H, W, 3), 128.0)
    for spacing, amp in ((96, 64), (48, 32), (24, 16), (12, 8), (6, 4)):
        for c in range(3):
            img[..., c] += amp * _value_noise(W, H, spacing, rng)
    y, x = np.mgrid[0:H, 0:W]
    for _ in range(n_edges):
        while True:
            nx, ny = (int(v) for v in rng.integers(-100, 101, size=2))
            if nx or ny:
                break
        px, py = int(rng.integers(0, W)), int(rng.integers(0, H))
        side = (x - px) * nx + (y - py) * ny > 0
        off = rng.integers(-50, 51, size=3)
        img[side] += off
    return _to_u8(img)


def content_voronoi_textures(W: int, H: int, rng: np.random.Generator, n_regions: int = 12) -> np.ndarray:
    """Voronoi regions, each a periodic texture, plus a gradient and noise."""
    sx = rng.integers(0, W, size=n_regions)
    sy = rng.integers(0, H, size=n_regions)
    y, x = np.mgrid[0:H, 0:W]
    best = np.full((H, W), np.iinfo(np.int64).max, dtype=np.int64)
    region = np.zeros((H, W), dtype=np.int32)
    for i in range(n_regions):
        d = (x - int(sx[i])).astype(np.int64) ** 2 + (y - int(sy[i])).astype(np.int64) ** 2
        closer = d < best
        best[closer] = d[closer]
        region[closer] = i
    img = np.zeros((H, W, 3), dtype=np.float64)
    for i in range(n_regions):
        sel = region == i
        if not sel.any():
            continue
        if rng.random() < 0.5:            # random u8 tile repeated
            px, py = (int(v) for v in rng.integers(4, 25, size=2))
            tile = rng.integers(0, 256, size=(py, px, 3)).astype(np.float64)
            img[sel] = tile[y[sel] % py, x[sel] % px]
        else:                              # integer-period triangle stripes
            per = int(rng.integers(4, 25))
            a, b = (int(v) for v in rng.integers(-3, 4, size=2))
            if a == 0 and b == 0:
                a = 1
            ph = ((a * x[sel] + b * y[sel]) % per).astype(np.float64)
            tri = np.abs(2.0 * ph / per - 1.0)   # triangle wave in [0, 1]
            c0 = rng.uniform(20, 120, size=3)
            c1 = rng.uniform(120, 235, size=3)
            img[sel] = c0[None, :] + (c1 - c0)[None, :] * tri[:, None]
    gx, gy = rng.uniform(-40, 40, size=2)
    img += (gx * (x / W) + gy * (y / H))[..., None]
    img += rng.integers(-3, 4, size=(H, W, 3))
    return _to_u8(img)


# -------------------------------------------------------------------- masks

def mask_ellipse_small() -> np.ndarray:
    """The 24x20 ellipse centred in a 128x96 frame."""
    y, x = np.mgrid[0:96, 0:128]
    inside = (2 * x - 127) ** 2 * 400 + (2 * y - 95) ** 2 * 576 <= 230400
    return inside.astype(np.uint8)


def mask_blobs(W: int, H: int, rng: np.random.Generator, area_frac: float, n_blobs: int,
               rad_lo: int, rad_hi: int, margin: int) -> np.ndarray:
    """Union of discs along random walks until the hole covers area_frac.

    Each blob starts in the central half of the frame; its discs stay at least
    ``margin`` pixels away from the border.
    """
    m = np.zeros((H, W), dtype=bool)
    target_total = int(area_frac * W * H)
    per_blob = [target_total // n_blobs] * n_blobs
    per_blob[-1] += target_total - sum(per_blob)
    area = 0
    for b in range(n_blobs):
        goal = area + per_blob[b]
        cx = int(rng.integers(W // 4, max(3 * W // 4, W // 4 + 1)))
        cy = int(rng.integers(H // 4, max(3 * H // 4, H // 4 + 1)))
        guard = 0
        while area < goal and guard < 100000:
            guard += 1
            rad = int(rng.integers(rad_lo, rad_hi + 1))
            rad = min(rad, (W - 1 - 2 * margin) // 2, (H - 1 - 2 * margin) // 2)
            lo_x, hi_x = margin + rad, W - 1 - margin - rad
            lo_y, hi_y = margin + rad, H - 1 - margin - rad
            cx = min(max(cx, lo_x), hi_x)
            cy = min(max(cy, lo_y), hi_y)
            x0, x1 = cx - rad, cx + rad + 1
            y0, y1 = cy - rad, cy + rad + 1
            yy, xx = np.mgrid[y0:y1, x0:x1]
            disc = (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
            area += int((disc & ~m[y0:y1, x0:x1]).sum())
            m[y0:y1, x0:x1] |= disc
            while True:
                dx, dy = (int(v) for v in rng.integers(-20, 21, size=2))
                if 100 <= dx * dx + dy * dy <= 400:
                    break
            cx += dx
            cy += dy
    return m.astype(np.uint8)


# ---------------------------------------------------------------- workloads

def small(seed: int = 1) -> Job:
    rng, = _rngs(seed, 1)
    return Job("small-128x96", content_gradient_rects(128, 96, rng), mask_ellipse_small(), 4)


def vga(seed: int = 2) -> Job:
    r_img, r_mask = _rngs(seed, 2)
    rgb = content_noise_edges(640, 480, r_img)
    mask = mask_blobs(640, 480, r_mask, 0.08, 1, 12, 30, 9)
    return Job("vga-640x480", rgb, mask, 4)


def hd(seed: int = 3, patch: int = 9, window: bool = False) -> Job:
    r_img, r_mask = _rngs(seed, 2)
    rgb = content_voronoi_textures(1920, 1080, r_img)
    mask = mask_blobs(1920, 1080, r_mask, 0.05, 1, 20, 60, 13)
    job = Job(f"hd-1920x1080-p{patch}-{'win' if window else 'full'}", rgb, mask, patch // 2)
    if window:
        job.search_mode, job.alpha = SEARCH_ALPHA, (1, 1)
    return job


def batch(seed: int = 4, n: int = 64, patch: int = 9) -> list[Job]:
    rngs = _rngs(seed, 1 + 2 * n)
    meta = rngs[0]
    jobs = []
    for i in range(n):
        W = int(meta.integers(320, 1281))
        H = int(meta.integers(240, 721))
        frac = float(meta.uniform(0.02, 0.10))
        nb = int(meta.integers(1, 4))
        r_img, r_mask = rngs[1 + 2 * i], rngs[2 + 2 * i]
        if i % 2 == 0:
            rgb = content_noise_edges(W, H, r_img)
        else:
            rgb = content_voronoi_textures(W, H, r_img)
        mask = mask_blobs(W, H, r_mask, frac, nb, 8, 30, patch)
        jobs.append(Job(f"batch{i}-{W}x{H}", rgb, mask, patch // 2))
    return jobs


def serving(seed: int = 5, n: int = 128, rate_per_s: float = 20.0,
            max_w: int = 2048, max_h: int = 1536) -> list[Job]:
    rngs = _rngs(seed, 1 + 2 * n)
    meta = rngs[0]
    t = 0.0
    jobs = []
    for i in range(n):
        t += float(meta.exponential(1.0 / rate_per_s))
        W = int(meta.integers(256, max_w + 1))
        H = int(meta.integers(256, max_h + 1))
        frac = float(meta.uniform(0.01, 0.10))
        nb = int(meta.integers(1, 4))
        patch = int(meta.choice([7, 9, 11]))
        r_img, r_mask = rngs[1 + 2 * i], rngs[2 + 2 * i]
        if i % 2 == 0:
            rgb = content_noise_edges(W, H, r_img)
        else:
            rgb = content_voronoi_textures(W, H, r_img)
        mask = mask_blobs(W, H, r_mask, frac, nb, 8, 30, patch)
        jobs.append(Job(f"serve{i}-{W}x{H}-p{patch}", rgb, mask, patch // 2, arrival_s=t))
    return jobs


def rescaled_arrivals(jobs: list[Job], rate_per_s: float, seed: int = 5) -> list[Job]:
    """Re-draws the arrival times of ``jobs`` for another Poisson rate."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[1])
    t = 0.0
    out = []
    for j in jobs:
        t += float(rng.exponential(1.0 / rate_per_s))
        out.append(dataclasses.replace(j, arrival_s=t))
    return out


# ------------------------------------------------------- small test inputs

def random_small(seed: int, W: int = 16, H: int = 16, hole: tuple | None = None,
                 levels: int = 256) -> Job:
    """Tiny random image with a rectangular or random hole, for brute force."""
    rng = np.random.default_rng(seed)
    rgb = rng.integers(0, levels, size=(H, W, 3)).astype(np.uint8)
    mask = np.zeros((H, W), dtype=np.uint8)
    if hole is None:
        x0, y0 = int(rng.integers(3, W - 6)), int(rng.integers(3, H - 6))
        w, h = int(rng.integers(2, 5)), int(rng.integers(2, 5))
        mask[y0:y0 + h, x0:x0 + w] = 1
    else:
        x0, y0, x1, y1 = hole
        mask[y0:y1, x0:x1] = 1
    return Job(f"rand{seed}-{W}x{H}", rgb, mask, 1)


def periodic_texture(seed: int, W: int, H: int, tile_w: int, tile_h: int, hole: tuple) -> tuple:
    """Noise-free periodic image (a random u8 tile repeated) with a hole."""
    rng = np.random.default_rng(seed)
    tile = rng.integers(0, 256, size=(tile_h, tile_w, 3)).astype(np.uint8)
    y, x = np.mgrid[0:H, 0:W]
    rgb = tile[y % tile_h, x % tile_w]
    mask = np.zeros((H, W), dtype=np.uint8)
    x0, y0, x1, y1 = hole
    mask[y0:y1, x0:x1] = 1
    return rgb, mask


WORKLOADS = {
    "small": small,
    "vga": vga,
    "hd": hd,
}


def mask_object(W: int, H: int, rng: np.random.Generator, obj_w: int, obj_h: int, margin: int) -> np.ndarray:
    """An irregular object whose bounding box is exactly obj_w x obj_h.

    The inscribed ellipse of the box (it touches all four sides) plus three
    to six discs centred in the middle half of the box, clipped to the box;
    the box is placed at a seeded position at least ``margin`` pixels from
    the border.
    """
    x0 = int(rng.integers(margin, W - margin - obj_w + 1))
    y0 = int(rng.integers(margin, H - margin - obj_h + 1))
    yy, xx = np.mgrid[0:obj_h, 0:obj_w]
    # (2x - (w-1))^2 h^2 + (2y - (h-1))^2 w^2 <= w^2 h^2
    a2, b2 = obj_w * obj_w, obj_h * obj_h
    inside = (2 * xx - (obj_w - 1)) ** 2 * b2 + (2 * yy - (obj_h - 1)) ** 2 * a2 <= a2 * b2
    for _ in range(int(rng.integers(3, 7))):
        cx = int(rng.integers(obj_w // 4, obj_w - obj_w // 4))
        cy = int(rng.integers(obj_h // 4, obj_h - obj_h // 4))
        rad = int(rng.integers(max(2, min(obj_w, obj_h) // 8), max(3, min(obj_w, obj_h) // 4) + 1))
        inside |= (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
    m = np.zeros((H, W), dtype=np.uint8)
    m[y0:y0 + obj_h, x0:x0 + obj_w] = inside
    return m


# name, width, height, object width, object height (Table 3)
PAPER_IMAGES = [
    ("WalkingMan", 512, 384, 78, 126),
    ("River", 480, 639, 59, 93),
    ("DivingMan", 576, 384, 155, 186),
    ("Hill", 1024, 550, 1024, 10),
]


def paper(name: str, seed: int = 6, patch: int = 9, alpha: tuple | None = None) -> Job:
    """Stand-in for one of the paper's photographs; alpha None = full search."""
    idx = [n for n, *_ in PAPER_IMAGES].index(name)
    _, W, H, ow, oh = PAPER_IMAGES[idx]
    r_img, r_mask = _rngs(seed * 16 + idx, 2)
    rgb = content_noise_edges(W, H, r_img)
    if ow >= W:   # a strip across the whole width
        y0 = int(r_mask.integers(H // 3, 2 * H // 3))
        mask = np.zeros((H, W), dtype=np.uint8)
        mask[y0:y0 + oh, :] = 1
    else:
        mask = mask_object(W, H, r_mask, ow, oh, 9)
    job = Job(f"{name}-{W}x{H}-p{patch}-" + ("full" if alpha is None else f"a{alpha[0]}/{alpha[1]}"),
              rgb, mask, patch // 2)
    if alpha is not None:
        job.search_mode, job.alpha = SEARCH_ALPHA, alpha
    return job
