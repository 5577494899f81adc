"""Seeded synthetic greyscale images shaped like the paper's workloads.

The paper measures on 512x512 8-bit greyscale photographs (Sec. 2, Sec. 4);
those images are not available, so every workload here is synthetic and
seeded.  This module draws pixels and nothing else: it holds none of the
encoder's or decoder's arithmetic, and both the CPU oracle's tests and the
GPU path consume exactly the bytes it returns.

Generators (all use ``numpy.random.Generator(PCG64(seed))``):

* ``noise_1f``       -- 1/f-spectrum Gaussian noise (power ~ f^-2), min-max
                        scaled to 0..255 and rounded.
* ``polygons``       -- star-shaped hard-edged polygons of constant grey,
                        painted over a base image in order (even-odd rule at
                        pixel centres).
* ``piecewise_smooth`` -- random quadratic patches on a Voronoi partition plus
                        Gaussian noise, rounded and clipped to 0..255.

Named workloads (``workload(name)``) fix sizes and seeds:

* ``c1``  64x64 1/f noise, seed 1.
* ``c2``  512x512 1/f noise + 8 polygons, seed 2.
* ``c3``  4096x4096 piecewise-smooth, 512 cells, sigma 4, seed 3.
* ``c4``  256 images, sides log-uniform in 128..2048 rounded to multiples of
          32, half noise / half piecewise-smooth, seed 4 (``SeedSequence``
          children, one per image).
* ``c5``  request pool for the serving loop: sides log-uniform in 64..4096
          rounded to multiples of 16, same mix, seed 5.
"""
from __future__ import annotations

import hashlib

import numpy as np
from scipy.spatial import cKDTree

__all__ = [
    "noise_1f", "polygons", "piecewise_smooth", "ramp", "flat",
    "c4_sides", "c4_images", "c5_sides", "c5_image", "workload", "sha256",
]


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def _to_u8_minmax(x: np.ndarray) -> np.ndarray:
    lo, hi = float(x.min()), float(x.max())
    if hi <= lo:
        return np.full(x.shape, 128, np.uint8)
    return np.rint((x - lo) * (255.0 / (hi - lo))).astype(np.uint8)


def noise_1f(h: int, w: int, seed, beta: float = 2.0) -> np.ndarray:
    """1/f noise: white N(0,1) -> FFT -> amplitude * |f|^(-beta/2), DC = 0
    -> real inverse FFT -> min-max to 0..255 -> rint."""
    rng = _rng(seed)
    white = rng.standard_normal((h, w))
    spec = np.fft.rfft2(white)
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.rfftfreq(w)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    spec = spec * f ** (-beta / 2.0)
    spec[0, 0] = 0.0
    field = np.fft.irfft2(spec, s=(h, w))
    return _to_u8_minmax(field)


def polygons(base: np.ndarray, count: int, seed) -> np.ndarray:
    """Paint ``count`` star-shaped polygons (3..8 vertices, radius 5..25 % of
    the shorter side, constant grey U{0..255}) over ``base`` in order."""
    rng = _rng(seed)
    img = base.copy()
    h, w = img.shape
    side = min(h, w)
    yc, xc = np.mgrid[0:h, 0:w]
    px = xc + 0.5
    py = yc + 0.5
    for _ in range(count):
        nv = int(rng.integers(3, 9))
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        rad = rng.uniform(0.05, 0.25) * side
        ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, nv))
        rr = rad * rng.uniform(0.5, 1.0, nv)
        vx = cx + rr * np.cos(ang)
        vy = cy + rr * np.sin(ang)
        grey = np.uint8(rng.integers(0, 256))
        inside = np.zeros((h, w), bool)
        j = nv - 1
        for i in range(nv):  # even-odd crossing test at pixel centres
            yi, yj, xi, xj = vy[i], vy[j], vx[i], vx[j]
            cond = (yi > py) != (yj > py)
            with np.errstate(divide="ignore", invalid="ignore"):
                xint = (xj - xi) * (py - yi) / (yj - yi) + xi
            inside ^= cond & (px < xint)
            j = i
        img[inside] = grey
    return img


def piecewise_smooth(h: int, w: int, seed, cells: int | None = None,
                     sigma: float = 4.0) -> np.ndarray:
    """Voronoi partition over ``cells`` uniform seeds; per cell a quadratic in
    coordinates normalised by the side, relative to the cell's seed:
    a ~ U(40, 215), linear ~ N(0, 60), quadratic ~ N(0, 120); plus N(0,
    sigma^2) noise; rint; clip to 0..255."""
    rng = _rng(seed)
    if cells is None:
        cells = max(16, int(round(512 * (h * w) / float(4096 * 4096))))
    side = float(max(h, w))
    sx = rng.uniform(0, w, cells)
    sy = rng.uniform(0, h, cells)
    a = rng.uniform(40.0, 215.0, cells)
    lin = rng.normal(0.0, 60.0, (cells, 2))
    quad = rng.normal(0.0, 120.0, (cells, 3))
    tree = cKDTree(np.stack([sx, sy], 1))
    out = np.empty((h, w), np.uint8)
    xs = np.arange(w, dtype=np.float64) + 0.5
    rows = max(1, (1 << 22) // max(w, 1))
    for y0 in range(0, h, rows):
        y1 = min(h, y0 + rows)
        gy, gx = np.meshgrid(np.arange(y0, y1, dtype=np.float64) + 0.5, xs,
                             indexing="ij")
        _, lab = tree.query(np.stack([gx.ravel(), gy.ravel()], 1), workers=-1)
        lab = lab.reshape(gx.shape)
        u = (gx - sx[lab]) / side
        v = (gy - sy[lab]) / side
        val = (a[lab] + lin[lab, 0] * u + lin[lab, 1] * v
               + quad[lab, 0] * u * u + quad[lab, 1] * u * v + quad[lab, 2] * v * v)
        val = val + rng.normal(0.0, sigma, val.shape)
        out[y0:y1] = np.clip(np.rint(val), 0, 255).astype(np.uint8)
    return out


def ramp(h: int, w: int) -> np.ndarray:
    """I[y][x] = 2x + 2y (needs h + w <= 128 to stay within 0..255)."""
    yy, xx = np.mgrid[0:h, 0:w]
    v = 2 * xx + 2 * yy
    if v.max() > 255:
        raise ValueError("ramp exceeds 8 bits")
    return v.astype(np.uint8)


def flat(h: int, w: int, value: int) -> np.ndarray:
    return np.full((h, w), value, np.uint8)


def _log_uniform_side(rng: np.random.Generator, lo: int, hi: int, mult: int) -> int:
    s = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    return int(max(lo, min(hi, mult * int(round(s / mult)))))


def c4_sides(n: int = 256, seed: int = 4):
    """Per-image (side, kind) for the batched workload: side log-uniform in
    128..2048 rounded to a multiple of 32; kind 0 = 1/f noise, 1 =
    piecewise-smooth, each with probability 1/2."""
    children = np.random.SeedSequence(seed).spawn(n)
    out = []
    for ss in children:
        rng = _rng(ss.spawn(1)[0])
        side = _log_uniform_side(rng, 128, 2048, 32)
        kind = int(rng.integers(0, 2))
        out.append((side, kind, ss))
    return out


def _mixed_image(side: int, kind: int, ss: np.random.SeedSequence) -> np.ndarray:
    img_ss = ss.spawn(2)[1]
    if kind == 0:
        return noise_1f(side, side, img_ss)
    return piecewise_smooth(side, side, img_ss)


def c4_images(n: int = 256, seed: int = 4):
    return [_mixed_image(s, k, ss) for (s, k, ss) in c4_sides(n, seed)]


def c5_sides(n: int = 512, seed: int = 5):
    """Request pool for serving: side log-uniform in 64..4096 rounded to a
    multiple of 16, same 50/50 generator mix."""
    children = np.random.SeedSequence(seed).spawn(n)
    out = []
    for ss in children:
        rng = _rng(ss.spawn(1)[0])
        side = _log_uniform_side(rng, 64, 4096, 16)
        kind = int(rng.integers(0, 2))
        out.append((side, kind, ss))
    return out


def c5_image(entry) -> np.ndarray:
    side, kind, ss = entry
    return _mixed_image(side, kind, ss)


def workload(name: str):
    """Return the image (or list of images) of a named workload."""
    if name == "c1":
        return noise_1f(64, 64, 1)
    if name == "c2":
        base = noise_1f(512, 512, 2)
        return polygons(base, 8, np.random.SeedSequence(2).spawn(1)[0])
    if name == "c3":
        return piecewise_smooth(4096, 4096, 3, cells=512, sigma=4.0)
    if name == "c4":
        return c4_images()
    raise KeyError(name)


def sha256(img: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(img).tobytes())
    return h.hexdigest()
