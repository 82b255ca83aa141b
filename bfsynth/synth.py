"""Seeded synthetic images standing in for the paper's test images.

The paper measures on natural 512x512 8-bit photographs and on a 256x256
black/white checkerboard (Section 4).  None of those files is available, so
each workload below is a seeded generator with the size, bit depth and
structure (flat regions, step edges, smooth ramps, additive noise) of the
workload it stands in for.  Every generator uses numpy's PCG64 with
``seed = 12030000 + config_index``; rounding is ``np.rint`` then clip.

Nothing here computes any part of the filter.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1203_0000

# Workload parameters.  sigma_s and radius in pixels; sigma_r and t_value in
# intensity units of the dtype; eps is the truncation tolerance.
CONFIGS = {
    1: dict(name="rect256_u8_global", H=256, W=256, dtype="u8", sigma_s=3.0, radius=9,
            sigma_r=30.0, eps=1e-3, t_mode="global", t_value=255.0, blur="iir_f32"),
    2: dict(name="grad512_u8_local", H=512, W=512, dtype="u8", sigma_s=10.0, radius=30,
            sigma_r=10.0, eps=1e-3, t_mode="local", t_value=0.0, blur="iir_f32"),
    3: dict(name="poly2048_u16_local", H=2048, W=2048, dtype="u16", sigma_s=8.0, radius=24,
            sigma_r=800.0, eps=1e-4, t_mode="local", t_value=0.0, blur="iir_f32"),
    4: dict(name="mosaic4096_f32_local", H=4096, W=4096, dtype="f32", sigma_s=16.0, radius=48,
            sigma_r=20.0, eps=1e-3, t_mode="local", t_value=0.0, blur="toeplitz_f16"),
    5: dict(name="batch64_u8_local", n_images=64, dtype="u8", eps=1e-3, t_mode="local",
            t_value=0.0, blur="auto"),
}


def _rng(cfg_index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + cfg_index))


def _finish(img: np.ndarray, hi: float, dtype) -> np.ndarray:
    return np.clip(np.rint(img), 0, hi).astype(dtype)


def gen_rect_u8(rng: np.random.Generator, H: int, W: int, n_rect: int = 24,
                noise: float = 10.0) -> np.ndarray:
    """Piecewise-constant axis-aligned rectangles on a random background, plus noise."""
    img = np.full((H, W), float(rng.integers(0, 256)))
    for _ in range(n_rect):
        y0, y1 = np.sort(rng.integers(0, H + 1, 2))
        x0, x1 = np.sort(rng.integers(0, W + 1, 2))
        img[y0:y1, x0:x1] = float(rng.integers(0, 256))
    img += rng.normal(0.0, noise, (H, W))
    return _finish(img, 255, np.uint8)


def gen_gradient_steps_u8(rng: np.random.Generator, H: int, W: int, n_steps: int = 16,
                          noise: float = 5.0) -> np.ndarray:
    """A linear ramp (about 40 to 200) in a random direction, random half-plane
    steps of +-U(20, 80), plus noise."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    a = rng.uniform(0.0, 2.0 * np.pi)
    d = np.cos(a) * xx + np.sin(a) * yy
    span = d.max() - d.min()
    d = (d - d.min()) / (span if span > 0 else 1.0)
    img = 40.0 + 160.0 * d
    for _ in range(n_steps):
        b = rng.uniform(0.0, 2.0 * np.pi)
        px, py = rng.uniform(0, W), rng.uniform(0, H)
        side = (np.cos(b) * (xx - px) + np.sin(b) * (yy - py)) > 0
        img += np.where(side, rng.choice([-1.0, 1.0]) * rng.uniform(20.0, 80.0), 0.0)
    img += rng.normal(0.0, noise, (H, W))
    return _finish(img, 255, np.uint8)


def _fill_polygon(mask_out: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> None:
    """Even-odd scanline fill of one polygon, sampled at pixel centres."""
    H, W = mask_out.shape
    yc = np.arange(H) + 0.5
    nv = len(xs)
    cuts = []
    for e in range(nv):
        xa, ya = xs[e], ys[e]
        xb, yb = xs[(e + 1) % nv], ys[(e + 1) % nv]
        if ya == yb:
            continue
        lo, hi = (ya, yb) if ya < yb else (yb, ya)
        inside = (yc >= lo) & (yc < hi)
        t = (yc - ya) / (yb - ya)
        cuts.append(np.where(inside, xa + t * (xb - xa), np.nan))
    if not cuts:
        return
    c = np.sort(np.stack(cuts, 0), axis=0)  # NaN sort last
    diff = np.zeros((H, W + 1), np.int32)
    rows = np.arange(H)
    for k in range(0, c.shape[0] - 1, 2):
        a, b = c[k], c[k + 1]
        ok = ~np.isnan(a) & ~np.isnan(b)
        a, b = np.where(ok, a, 0.0), np.where(ok, b, 0.0)
        s = np.clip(np.ceil(a - 0.5), 0, W).astype(np.int64)
        t = np.clip(np.floor(b - 0.5) + 1, 0, W).astype(np.int64)
        ok &= t > s
        np.add.at(diff, (rows[ok], s[ok]), 1)
        np.add.at(diff, (rows[ok], t[ok]), -1)
    mask_out |= (np.cumsum(diff, axis=1)[:, :W] % 2) == 1


def gen_polygons_u16(rng: np.random.Generator, H: int, W: int, n_poly: int = 64,
                     noise: float = 300.0) -> np.ndarray:
    """Random polygons (3-8 vertices) painted in order on a random background, plus noise."""
    img = np.full((H, W), float(rng.integers(0, 65536)))
    for _ in range(n_poly):
        nv = int(rng.integers(3, 9))
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        rad = rng.uniform(0.05, 0.35) * min(H, W)
        ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
        rr = rad * rng.uniform(0.4, 1.0, nv)
        xs, ys = cx + rr * np.cos(ang), cy + rr * np.sin(ang)
        m = np.zeros((H, W), bool)
        _fill_polygon(m, xs, ys)
        img[m] = float(rng.integers(0, 65536))
    img += rng.normal(0.0, noise, (H, W))
    return _finish(img, 65535, np.uint16)


def gen_mosaic_f32(rng: np.random.Generator, H: int, W: int, n_tiles: int = 256,
                   noise: float = 8.0) -> np.ndarray:
    """Recursive random rectangle splits, each tile U[0,255], plus noise; clipped, not rounded."""
    tiles = [(0, 0, H, W)]
    while len(tiles) < n_tiles:
        i = int(rng.integers(len(tiles)))
        y0, x0, y1, x1 = tiles[i]
        if y1 - y0 < 4 and x1 - x0 < 4:
            if all((t[2] - t[0] < 4 and t[3] - t[1] < 4) for t in tiles):
                break
            continue
        tiles.pop(i)
        if (y1 - y0) >= (x1 - x0):
            c = int(rng.integers(y0 + 1, y1))
            tiles += [(y0, x0, c, x1), (c, x0, y1, x1)]
        else:
            c = int(rng.integers(x0 + 1, x1))
            tiles += [(y0, x0, y1, c), (y0, c, y1, x1)]
    img = np.zeros((H, W))
    for (y0, x0, y1, x1) in tiles:
        img[y0:y1, x0:x1] = rng.uniform(0.0, 255.0)
    img += rng.normal(0.0, noise, (H, W))
    return np.clip(img, 0.0, 255.0).astype(np.float32)


def gen_checker_u8(H: int = 256, W: int = 256, square: int = 32) -> np.ndarray:
    """Black (0) and white (255) squares, the kind of image the paper calls Checker."""
    yy, xx = np.mgrid[0:H, 0:W]
    return (((yy // square + xx // square) % 2) * 255).astype(np.uint8)


def gen_random(seed: int, H: int, W: int, dtype: str = "u8", kind: str = "mixed") -> np.ndarray:
    """Small seeded images for parity sweeps (any shape, incl. 1xN and Nx1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hi = {"u8": 255.0, "u16": 65535.0, "f32": 255.0}[dtype]
    if kind == "noise":
        img = rng.uniform(0, hi, (H, W))
    elif kind == "const":
        img = np.full((H, W), rng.uniform(0, hi))
    elif kind == "step":
        img = np.where(np.arange(W)[None, :] < W // 2, 0.2 * hi, 0.8 * hi) * np.ones((H, 1))
    else:
        img = np.full((H, W), rng.uniform(0, hi))
        for _ in range(6):
            y0, y1 = np.sort(rng.integers(0, H + 1, 2))
            x0, x1 = np.sort(rng.integers(0, W + 1, 2))
            img[y0:y1, x0:x1] = rng.uniform(0, hi)
        img += rng.normal(0, 0.03 * hi, (H, W))
    if dtype == "u8":
        return _finish(img, 255, np.uint8)
    if dtype == "u16":
        return _finish(img, 65535, np.uint16)
    return np.clip(img, 0, hi).astype(np.float32)


def config_image(idx: int) -> np.ndarray:
    """The seeded input image of workload ``idx`` (1-4)."""
    c = CONFIGS[idx]
    rng = _rng(idx)
    if idx == 1:
        return gen_rect_u8(rng, c["H"], c["W"])
    if idx == 2:
        return gen_gradient_steps_u8(rng, c["H"], c["W"])
    if idx == 3:
        return gen_polygons_u16(rng, c["H"], c["W"])
    if idx == 4:
        return gen_mosaic_f32(rng, c["H"], c["W"])
    raise ValueError(idx)


def batch_images(n: int | None = None):
    """Workload 5: uneven-size 8-bit images with per-image sigma_s, sigma_r.

    Returns a list of (image, sigma_s, sigma_r).  Sizes are drawn uniformly from
    128..1024 per axis; content alternates the rectangle and gradient generators.
    """
    c = CONFIGS[5]
    n = c["n_images"] if n is None else n
    rng = _rng(5)
    out = []
    for i in range(n):
        H = int(rng.integers(128, 1025))
        W = int(rng.integers(128, 1025))
        ss = float(rng.uniform(2.0, 16.0))
        sr = float(rng.uniform(10.0, 60.0))
        sub = np.random.Generator(np.random.PCG64(SEED_BASE + 5000 + i))
        img = gen_rect_u8(sub, H, W) if i % 2 == 0 else gen_gradient_steps_u8(sub, H, W)
        out.append((img, ss, sr))
    return out
