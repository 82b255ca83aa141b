"""The tile-skipping rule of the range stage, checked on the CPU against the
oracle's Algorithm 1 (max filter map and T):

* the lower bound -- the largest (max - min) over the b x b sub-blocks of
  the 32 x 32 tiles, b the largest power of two <= min(R + 1, 32) -- never
  exceeds T;
* every tile the rule skips (largest maximum of the tiles within reach of
  its outputs' windows minus its own minimum <= the bound) holds no output
  whose window maximum minus f exceeds the bound;

so max(bound, the other tiles' maxima) is T.  Images with flat regions,
ramps, steps, spikes and noise, ragged sizes, R from 1 to 48."""
import math

import numpy as np
import pytest

import oracle as o
from bfsynth import gen_random

TILE = 32


def _blocks(f, b):
    H, W = f.shape
    ny, nx = -(-H // b), -(-W // b)
    g = np.full((ny * b, nx * b), np.nan)
    g[:H, :W] = f
    g = g.reshape(ny, b, nx, b)
    return np.nanmax(g, axis=(1, 3)), np.nanmin(g, axis=(1, 3))


def _rule(f, R):
    b = 1
    while 2 * b <= min(R + 1, TILE):
        b *= 2
    smx, smn = _blocks(f, b)
    lb = float((smx - smn).max())
    tmx, tmn = _blocks(f, TILE)
    rt = math.ceil(R / TILE)
    ny, nx = tmx.shape
    skip = np.zeros((ny, nx), bool)
    for ty in range(ny):
        for tx in range(nx):
            reach = tmx[max(0, ty - rt):ty + rt + 1, max(0, tx - rt):tx + rt + 1].max()
            skip[ty, tx] = reach - tmn[ty, tx] <= lb
    return lb, skip


def _images():
    rng = np.random.default_rng(5)
    H, W = 150, 203
    yy, xx = np.mgrid[0:H, 0:W]
    ramp = 30.0 + 0.4 * xx + 0.25 * yy
    steps = ramp.copy()
    for _ in range(5):
        steps[rng.integers(0, H):, rng.integers(0, W):] += rng.uniform(-30, 30)
    spikes = np.full((H, W), 90.0)
    spikes[rng.integers(0, H, 6), rng.integers(0, W, 6)] = rng.uniform(0, 255, 6)
    pair = np.full((H, W), 100.0)
    pair[70, 60], pair[70, 100] = 3.0, 250.0
    noisy = gen_random(9, H, W, "u8", "mixed").astype(np.float64)
    return [ramp, steps, spikes, pair, noisy]


@pytest.mark.parametrize("R", [1, 2, 5, 15, 16, 31, 40, 48])
def test_skip_rule_is_exact(R):
    n_skipped = 0
    for f in _images():
        T, Mx = o.range_T(f, R, return_map=True)
        lb, skip = _rule(f, R)
        assert lb <= T
        local = Mx - f
        H, W = f.shape
        best = lb
        for ty, tx in zip(*np.nonzero(skip)):
            tile = local[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE]
            assert tile.max() <= lb
        for ty, tx in zip(*np.nonzero(~skip)):
            best = max(best, local[ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE].max())
        assert best == T
        n_skipped += int(skip.sum())
    if R >= 15:
        assert n_skipped > 0  # the rule does skip tiles on these images
