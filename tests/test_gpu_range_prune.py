"""GPU: the range stage's tile skipping leaves T exact (Algorithm 1).

The tile kernel skips 32 x 32 output tiles whose bound (largest tile maximum
within reach of the window minus the tile's own minimum) does not exceed a
lower bound of T taken from the sub-blocks of the tiles (their max - min).
These images put the maximising pair across tiles and sub-blocks, on flat or
smooth backgrounds where most tiles are skipped, so T must come from the few
tiles computed in full or equal the lower bound itself.  T is compared with
the oracle's Algorithm 1 exactly, for every dtype and both tile-kernel sizes.
Single images take the statistics pass from 1024 tiles up (the images here
are about 1 MP); batches always do (the batch tests use small images).
"""
import numpy as np
import pytest

import oracle as o

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _T(img, dtype, R):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    sr = 20.0 * (257.0 if dtype == "u16" else 1.0)
    plan = Plan.create(make_params(H, W, dtype, sigma_s=2.0, sigma_r=sr, radius=R, t_mode="local"))
    T = plan.dynamic_range(torch.from_numpy(np.ascontiguousarray(img)).to("cuda"))
    plan.close()
    return T


def _cast(img, dtype):
    return img.astype({"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[dtype])


def _scale(dtype):
    return 257.0 if dtype == "u16" else 1.0


@pytest.mark.parametrize("R", [2, 7, 15, 31, 40, 48])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_pair_across_tiles(R, dtype):
    """Flat background, one dark and one bright pixel R apart in different
    tiles: T (their difference) exceeds every sub-block's range, so only
    the tiles around the dark pixel can hold it."""
    H, W = 1030, 1057
    img = np.full((H, W), 100.0)
    y, x = 700, 600
    img[y, x] = 3.0
    img[y, x + R] = 250.0
    img = _cast(img * _scale(dtype), dtype)
    T = _T(img, dtype, R)
    ref = o.range_T(img.astype(np.float64), R)
    print(f"[prune] pair R={R} {dtype} T={T} oracle={ref}", flush=True)
    assert T == ref == (250.0 - 3.0) * _scale(dtype)


@pytest.mark.parametrize("R", [1, 3, 16, 32, 47])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_smooth_background_with_features(R, dtype):
    """A slow ramp (small local ranges everywhere) with a few steps and
    spikes at seeded places, ragged size."""
    rng = np.random.default_rng(1000 + R)
    H, W = 1041, 1029
    yy, xx = np.mgrid[0:H, 0:W]
    img = 40.0 + 0.1 * xx + 0.07 * yy
    for _ in range(6):
        y0, x0 = rng.integers(0, H), rng.integers(0, W)
        img[y0:y0 + 9, x0:x0 + 13] += rng.uniform(-35, 35)
    for _ in range(8):
        img[rng.integers(0, H), rng.integers(0, W)] = rng.uniform(0, 255)
    img = np.clip(np.rint(img), 0, 255)
    if dtype == "f32":
        img = img + rng.uniform(0.0, 0.5, img.shape)  # fractional values
    img = _cast(img * _scale(dtype), dtype)
    T = _T(img, dtype, R)
    ref = o.range_T(img.astype(np.float64), R)
    print(f"[prune] ramp R={R} {dtype} T={T} oracle={ref}", flush=True)
    assert T == ref


@pytest.mark.parametrize("R", [4, 31, 48])
def test_checkerboard(R):
    """A 0/255 checkerboard of 16-pixel squares.  R = 4: the 4 x 4
    sub-blocks lie inside squares (lower bound 0), every tile is computed.
    R >= 31: a tile's sub-block holds both values, the bound is the full
    range and every tile is skipped, so T is the bound itself."""
    H, W = 1030, 1025
    yy, xx = np.mgrid[0:H, 0:W]
    img = (((yy // 16) + (xx // 16)) % 2 * 255).astype(np.uint8)
    T = _T(img, "u8", R)
    assert T == o.range_T(img.astype(np.float64), R) == 255.0


@pytest.mark.parametrize("R", [5, 33])
def test_float_many_binades(R):
    """Float samples from 1e-6 to 250 (several binades) on a flat
    background, with the extreme pair in different tiles."""
    rng = np.random.default_rng(77 + R)
    H, W = 1024, 1040
    img = np.full((H, W), 120.0, dtype=np.float64)
    img[rng.integers(0, H, 20), rng.integers(0, W, 20)] = rng.uniform(0.0, 250.0, 20)
    img[rng.integers(0, H, 20), rng.integers(0, W, 20)] = 10.0 ** rng.uniform(-6, -2, 20)
    img = img.astype(np.float32)
    T = _T(img, "f32", R)
    assert T == o.range_T(img.astype(np.float64), R)


def test_bound_cleared_between_calls():
    """A call with a large bound, then images whose T is small: each gets
    its own T (the lower bounds are cleared when T is published)."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W, R = 1040, 1050, 40
    plan = Plan.create(make_params(H, W, "u8", sigma_s=2.0, sigma_r=20.0, radius=R, t_mode="local"))
    yy, xx = np.mgrid[0:H, 0:W]
    imgs = [((xx // 8) % 2 * 255).astype(np.uint8),
            np.full((H, W), 9, np.uint8),
            (50 + (xx // 40)).astype(np.uint8)]
    imgs[1][60, 70] = 13
    for img in imgs + imgs[::-1]:
        T = plan.dynamic_range(torch.from_numpy(img).to("cuda"))
        assert T == o.range_T(img.astype(np.float64), R)
    plan.close()


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_batch_images(dtype):
    """Grouped launches (statistics always on): small structured images with
    radii on both tile-kernel sizes; each report's T against the oracle."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    rng = np.random.default_rng(31)
    imgs, params = [], []
    for i, (H, W, R) in enumerate([(150, 211, 40), (97, 300, 3), (260, 130, 48), (64, 64, 16), (200, 190, 31),
                                   (33, 47, 9)]):
        yy, xx = np.mgrid[0:H, 0:W]
        img = 60.0 + 0.2 * xx + 0.1 * yy
        img[rng.integers(0, H), rng.integers(0, W)] = rng.uniform(0, 255)
        if i % 2:
            img[H // 2, W // 3], img[H // 2, min(W - 1, W // 3 + R)] = 2.0, 253.0
        img = _cast(np.clip(img, 0, 255), dtype)
        imgs.append(img)
        params.append(make_params(H, W, dtype, sigma_s=2.0, sigma_r=20.0, radius=R, t_mode="local"))
    plan = Plan.create(params)
    _, reps = plan.filter_batch([torch.from_numpy(im).to("cuda") for im in imgs])
    torch.cuda.synchronize()
    for img, p, rep in zip(imgs, params, reps):
        assert rep["T"] == o.range_T(img.astype(np.float64), p.radius)
    plan.close()
