"""CPU model of the one-launch dynamic-range kernel, checked against the oracle.

The kernel computes Algorithm 1 (row then column MAX-FILTER, T = max over
pixels of window maximum minus the pixel, Prop. 2.1 with the sign read from
its proof) on 32 x 32 output blocks with an R-pixel halo.  For 2R + 1 >= 32
each line of 32 + 2R samples x gives output j the window
[j, j+2R] = [j, 30] u [31, 2R] u [2R+1, 2R+j]: a suffix maximum over lanes,
a maximum common to every window (entered as lane 31's sample of the suffix
scan), and a prefix maximum; lanes whose piece is empty read a sample every
window holds instead of a masked value.  Narrower windows take a direct
maximum.  Samples are compared through integer keys: the value itself for 8-
and 16-bit input (out-of-image samples 0), the sign-folded float bit pattern
for float input (non-finite and out-of-image samples -inf).

This model restates that decomposition lane by lane in NumPy, so that a
mistake in it (a wrong piece boundary, a duplicate read outside every window,
a key that does not order like the samples) fails here, on the CPU.  It
shares no code with the library or the oracle; the expected T is the oracle's.
"""
import numpy as np
import pytest

import oracle as o
from bfsynth import gen_random

TW = TH = 32


def keys(v, dtype):
    """Integer keys that order like the samples."""
    if dtype == "f32":
        v = np.where(np.isfinite(v), v, -np.inf).astype(np.float32)
        bits = v.view(np.int32).astype(np.int64)
        return np.where(bits < 0, bits ^ 0x7FFFFFFF, bits)
    return v.astype(np.int64)


def unkey(k, dtype):
    if dtype == "f32":
        k = np.asarray(k, dtype=np.int64)
        bits = np.where(k < 0, k ^ 0x7FFFFFFF, k).astype(np.int32)
        return bits.view(np.float32).astype(np.float64)
    return np.asarray(k, dtype=np.float64)


def line_max(x, R):
    """Window maxima of outputs j in [0, 32) over samples x[j .. j+2R]
    (len(x) = 32 + 2R), the way a half-wave forms them."""
    j = np.arange(32)
    if R < 16:
        return np.array([x[i:i + 2 * R + 1].max() for i in range(32)])
    nc = 2 * R - 30  # samples [31, 2R]
    c = x[31 + np.minimum(j, nc - 1)]
    if nc > 32:
        c = np.maximum(c, x[63 + np.minimum(j, nc - 33)])
    if nc > 64:
        c = np.maximum(c, x[95 + np.minimum(j, nc - 65)])
    C = c.max()
    a = x[j].copy()
    a[31] = C
    S = np.maximum.accumulate(a[::-1])[::-1]  # suffix over lanes k >= j
    P = np.maximum.accumulate(x[2 * R + j])   # prefix over lanes k <= j
    return np.maximum(S, P)


def model_T(img, R, dtype):
    """T and the window-maximum map, block by block."""
    H, W = img.shape
    pad = -np.inf if dtype == "f32" else 0
    T = 0.0
    Mx = np.full((H, W), np.nan)
    for y0 in range(0, H, TH):
        for x0 in range(0, W, TW):
            L, Lc = TH + 2 * R, TW + 2 * R
            reg = np.full((L, Lc), pad, dtype=np.float64)
            ys, xs = y0 - R, x0 - R
            ya, yb = max(ys, 0), min(ys + L, H)
            xa, xb = max(xs, 0), min(xs + Lc, W)
            reg[ya - ys:yb - ys, xa - xs:xb - xs] = img[ya:yb, xa:xb]
            k = keys(reg, dtype)
            rm = np.stack([line_max(k[e], R) for e in range(L)])     # L x 32
            out = np.stack([line_max(rm[:, c], R) for c in range(TW)], axis=1)  # 32 x 32
            for jy in range(TH):
                for jx in range(TW):
                    y, x = y0 + jy, x0 + jx
                    if y < H and x < W:
                        Mx[y, x] = unkey(out[jy, jx], dtype)
                        d = Mx[y, x] - float(img[y, x])
                        if d > T:
                            T = d
    return T, Mx


CASES = [  # (H, W, R)
    (1, 1, 6), (1, 70, 40), (70, 1, 17), (33, 65, 1), (37, 45, 15), (40, 41, 16),
    (50, 70, 30), (45, 52, 31), (66, 35, 32), (40, 90, 33), (70, 60, 47), (75, 80, 48),
]


@pytest.mark.parametrize("H,W,R", CASES)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_tile_model_matches_oracle_T(H, W, R, dtype):
    """Every pixel's window maximum, and T, equal the oracle's exactly (a
    window that misses or adds a sample changes the map somewhere)."""
    img = gen_random(900 + H + 7 * W + R, H, W, dtype=dtype)
    T, Mx = model_T(img, R, dtype)
    T_ref, Mx_ref = o.range_T(img.astype(np.float64), R, return_map=True)
    assert np.array_equal(Mx, Mx_ref)
    assert T == T_ref


def distinct_image(seed, H, W, dtype):
    """All values distinct (a shuffled ramp), so that every window has a
    unique maximum and a window missing one sample changes the map wherever
    that sample was the maximum."""
    v = np.random.default_rng(seed).permutation(H * W).reshape(H, W)
    if dtype == "u16":
        return v.astype(np.uint16)
    return (v.astype(np.float32) * 0.37 - 1000.0).astype(np.float32)


@pytest.mark.parametrize("H,W,R", CASES)
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_tile_model_distinct_values(H, W, R, dtype):
    img = distinct_image(1700 + H + 3 * W + R, H, W, dtype)
    T, Mx = model_T(img, R, dtype)
    T_ref, Mx_ref = o.range_T(img.astype(np.float64), R, return_map=True)
    assert np.array_equal(Mx, Mx_ref)
    assert T == T_ref


@pytest.mark.parametrize("R", [3, 8, 15, 16, 24, 31, 32, 33, 47, 48])
def test_tile_model_single_spike_sweep(R):
    """One bright sample on low noise, moved along a row over every column of
    the image and down a column over every row: each window holding it must
    report it, so every sample offset each line piece reads is exercised in
    the row pass and in the column pass."""
    rng = np.random.default_rng(2100 + R)
    H, W = 24, 2 * 32 + 2
    base = rng.integers(0, 100, (H, W)).astype(np.uint16)
    spots = [(5, xs) for xs in range(W)] + [(ys, 40) for ys in range(H)]
    for ys, xs in spots:
        img = base.copy()
        img[ys, xs] = 60000
        T, Mx = model_T(img, R, "u16")
        T_ref, Mx_ref = o.range_T(img.astype(np.float64), R, return_map=True)
        assert np.array_equal(Mx, Mx_ref), (ys, xs)
        assert T == T_ref


def test_keys_order_like_floats():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(2000).astype(np.float32) * 100,
                        np.array([0.0, -0.0, 1e-30, -1e-30, 3e38, -3e38], np.float32)])
    k = keys(v, "f32")
    i, j = rng.integers(0, len(v), (2, 20000))
    fi, fj = v[i].astype(np.float64), v[j].astype(np.float64)
    strict = fi != fj
    assert np.array_equal((k[i] > k[j])[strict], (fi > fj)[strict])
    assert np.array_equal(unkey(k, "f32"), v.astype(np.float64))
    assert keys(np.array([np.nan, np.inf, -np.inf], np.float32), "f32").max() == keys(
        np.array([-np.inf], np.float32), "f32")[0]
