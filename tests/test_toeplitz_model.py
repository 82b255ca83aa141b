"""CPU model of the Toeplitz MFMA kernels' index arithmetic.

The model replays, lane by lane, the tile staging, the 16x16x32 fragment
layout, the Z store/load addressing (left pad R mod 8, 8-element vectors)
and the combine of the two kernels in FP64, asserting that every LDS and
global access stays inside its buffer.  Its output must equal the oracle's
Algorithm 2 with the FIR operator up to rounding; the GPU tests then compare
the kernels themselves with the oracle.
"""
import math

import numpy as np
import pytest

import oracle

LDS_MAX = 156 * 1024
LDS_PREF = 78 * 1024


def v_cols(split):
    return 16 if split else 32


def h_cols(split):
    return 64 if split else 128


def tap_bytes(split, nks):
    return (2 if split else 1) * nks * 64 * 16


def v_lds(split, rows, nks):
    Kp = rows - 16 + 32 * nks + 8
    return tap_bytes(split, nks) + (2 if split else 1) * 4 * v_cols(split) * Kp * 2


def h_lds(split, nks):
    Kp = h_cols(split) - 16 + 32 * nks + 8
    return tap_bytes(split, nks) + (2 if split else 1) * 4 * 16 * Kp * 2


def shape(split, R, H):
    """Tallest vertical tile within the preferred LDS budget, else the whole LDS."""
    nks = (16 + 2 * R + 31) // 32
    if nks > 8:
        return None
    top = min(256, (H + 15) // 16 * 16)
    rows = None
    for budget in (LDS_PREF, LDS_MAX):
        for r in range(top, 15, -16):
            if v_lds(split, r, nks) <= budget:
                rows = r
                break
        if rows:
            break
    if rows is None or h_lds(split, nks) > LDS_MAX:
        return None
    nty = (H + rows - 1) // rows
    rows = ((H + 15) // 16 + nty - 1) // nty * 16
    return nks, rows


def tap_matrix(w, R, nks):
    """T[i][t] = w[t - i] on the band, as the lanes' fragments build it."""
    T = np.zeros((16, 32 * nks))
    for ks in range(nks):
        for lane in range(64):
            i = lane & 15
            for j in range(8):
                d = 32 * ks + 8 * (lane >> 4) + j - i
                if 0 <= d <= 2 * R:
                    T[i, 32 * ks + 8 * (lane >> 4) + j] = w[d]
    return T


def mfma_product(a_at, b_at, nks):
    """D (16x16) of nks chained 16x16x32 products whose lane fragments are read
    through a_at(lane, ks) and b_at(lane, ks) (each returns 8 values)."""
    D = np.zeros((16, 16))
    for ks in range(nks):
        A = np.zeros((16, 32))
        B = np.zeros((32, 16))
        for lane in range(64):
            g, r = lane >> 4, lane & 15
            A[r, 8 * g:8 * g + 8] = a_at(lane, ks)
            B[8 * g:8 * g + 8, r] = b_at(lane, ks)
        D += A @ B
    return D


def model(f, planes, sigma_s, R, split, K, coef_phase):
    """planes: (K, 4, H, W) scaled planes per pair; coef_phase(k) -> (c', cos, sin)
    images.  Returns the filtered image (center and scale applied by caller)."""
    H, W = f.shape
    nks, rows = shape(split, R, H)
    w = np.exp(-((np.arange(2 * R + 1) - R) ** 2) / (2.0 * sigma_s ** 2))
    padl = R & 7
    zpitch = (W + padl + 7) // 8 * 8
    zplane = H * zpitch
    Z = np.full(K * 4 * zplane, np.nan)
    cv = v_cols(split)
    # vertical kernel
    Kl = rows - 16 + 32 * nks
    Kp = Kl + 8
    lds_elems = (v_lds(split, rows, nks) - tap_bytes(split, nks)) // 2 // (2 if split else 1)
    for kl in range(K):
        for by in range((H + rows - 1) // rows):
            for bx in range((W + cv - 1) // cv):
                x0, y0 = bx * cv, by * rows
                Bh = np.full(lds_elems, np.nan)
                for it in range((Kl // 8) * cv):
                    c, s = it % cv, it // cv
                    x = x0 + c
                    base = (np.arange(4) * cv + c) * Kp + 8 * s
                    assert base.max() + 8 <= lds_elems
                    for j in range(8):
                        y = y0 - R + 8 * s + j
                        val = planes[kl, :, y, x] if (0 <= y < H and x < W) else np.zeros(4)
                        Bh[base + j] = val
                for cb in range((rows // 16) * (cv // 16)):
                    mb, nb = cb % (rows // 16), cb // (rows // 16)
                    Tm = tap_matrix(w, R, nks)
                    for p in range(4):
                        def a_at(lane, ks):
                            return Tm[lane & 15, 32 * ks + 8 * (lane >> 4):32 * ks + 8 * (lane >> 4) + 8]

                        def b_at(lane, ks):
                            px = nb * 16 + (lane & 15)
                            o = (p * cv + px) * Kp + 16 * mb + 8 * (lane >> 4) + 32 * ks
                            assert o + 8 <= lds_elems
                            v = Bh[o:o + 8]
                            assert not np.isnan(v).any(), "read of unstaged LDS"
                            return v

                        # operands swapped: A = column fragments, B = taps -> D'[x][y]
                        Dt = mfma_product(b_at, a_at, nks)
                        for lane in range(64):
                            y = y0 + 16 * mb + (lane & 15)
                            xs = x0 + nb * 16 + 4 * (lane >> 4)
                            if y >= H or xs >= W:
                                continue
                            for i in range(4):
                                if xs + i < W:
                                    o = (kl * 4 + p) * zplane + y * zpitch + padl + xs + i
                                    assert 0 <= o < Z.size
                                    Z[o] = Dt[4 * (lane >> 4) + i, lane & 15]
    # horizontal kernel
    ch = h_cols(split)
    Klh = ch - 16 + 32 * nks
    Kph = Klh + 8
    lds_h = (h_lds(split, nks) - tap_bytes(split, nks)) // 2 // (2 if split else 1)
    P = np.zeros((H, W))
    Q = np.zeros((H, W))
    Tm = tap_matrix(w, R, nks)
    for by in range((H + 15) // 16):
        for bx in range((W + ch - 1) // ch):
            x0, y0 = bx * ch, by * 16
            zc0 = x0 - R + padl
            assert zc0 % 8 == 0
            for kl in range(K):
                Ah = np.full(lds_h, np.nan)
                nvec = Klh // 8
                for it in range(4 * 16 * nvec):
                    v, rr = it % nvec, it // nvec
                    p, r = rr // 16, rr % 16
                    y = y0 + r
                    zc = zc0 + 8 * v
                    vals = np.zeros(8)
                    if y < H and zc + 8 > padl and zc < padl + W:
                        src = (kl * 4 + p) * zplane + y * zpitch + zc
                        assert 0 <= zc and zc + 8 <= zpitch and src % 8 == 0
                        vals = Z[src:src + 8].copy()
                        for j in range(8):
                            if zc + j < padl or zc + j >= padl + W:
                                vals[j] = 0.0
                        assert not np.isnan(vals).any(), "load of unwritten Z"
                    o = rr * Kph + 8 * v
                    assert o + 8 <= lds_h
                    Ah[o:o + 8] = vals
                cp, cimg, simg = coef_phase(kl)
                for nb in range(ch // 16):
                    acc = []
                    for p in range(4):
                        def a_at(lane, ks):
                            o = (p * 16 + (lane & 15)) * Kph + 16 * nb + 8 * (lane >> 4) + 32 * ks
                            assert o + 8 <= lds_h
                            return Ah[o:o + 8]

                        def b_at(lane, ks):
                            return Tm[lane & 15, 32 * ks + 8 * (lane >> 4):32 * ks + 8 * (lane >> 4) + 8]

                        acc.append(mfma_product(a_at, b_at, nks))
                    for lane in range(64):
                        x = x0 + nb * 16 + (lane & 15)
                        for i in range(4):
                            y = y0 + 4 * (lane >> 4) + i
                            if y >= H or x >= W:
                                continue
                            r, n = 4 * (lane >> 4) + i, lane & 15
                            c, s = cimg[y, x], simg[y, x]
                            P[y, x] += cp * (c * acc[0][r, n] + s * acc[1][r, n])
                            Q[y, x] += cp * (c * acc[2][r, n] + s * acc[3][r, n])
    return P, Q


def table(sigma_r, eps, T, rng8=255.0):
    N = oracle.order(T, sigma_r)
    M = oracle.trunc_rule(N, sigma_r * 255.0 / rng8, eps)
    pairs = []
    for n in range(M, (N + 1) // 2):
        pairs.append((2 * n - N, 2.0 * oracle.coef(N, n)))
    if N % 2 == 0:
        pairs.append((0, oracle.coef(N, N // 2)))
    return N, M, pairs


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("H,W,R,sigma_s", [(37, 150, 5, 2.0), (70, 45, 13, 4.5), (20, 20, 0, 0.8),
                                           (290, 40, 3, 1.0)])
def test_model_matches_oracle_fir(split, H, W, R, sigma_s):
    rng = np.random.default_rng(1234 + H + R)
    yy, xx = np.mgrid[0:H, 0:W]
    f = np.clip(np.round(60 + 100 * (xx / W) + 40 * (yy > H // 2) + rng.normal(0, 8, (H, W))), 0, 255)
    sigma_r, eps = 20.0, 1e-3
    ref = oracle.algorithm2(f, "fir", sigma_s, R, sigma_r, eps, 255.0, True)
    N, M, pairs = table(sigma_r, eps, ref["T"])
    assert (N, M) == (ref["N"], ref["M"])
    center = 127.5
    alpha = 1.0 / (math.sqrt(N) * sigma_r)
    K = len(pairs)
    planes = np.zeros((K, 4, H, W))
    cs = []
    for k, (m, c) in enumerate(pairs):
        th = m * alpha * f
        co, si = np.cos(th), np.sin(th)
        d = (f - center) / center
        planes[k] = [d * co, d * si, co, si]
        cs.append((c, co, si))
    P, Q = model(f, planes, sigma_s, R, split, K, lambda k: cs[k])
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(Q > 0, center + center * P / Q, f)
    assert int((Q <= 0).sum()) == ref["n_nonpos"]
    assert np.abs(out - ref["out"]).max() < 1e-9


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("H,W,R", [(4096, 4096, 48), (512, 512, 30), (2048, 2048, 24), (1, 1, 0), (17, 3000, 72),
                                   (300, 200, 120)])
def test_extreme_tiles_in_bounds(split, H, W, R):
    """Address ranges of the first and last tiles of large launches."""
    nks, rows = shape(split, R, H)
    assert v_lds(split, rows, nks) <= LDS_MAX and h_lds(split, nks) <= LDS_MAX
    assert rows % 16 == 0 and 16 <= rows <= max(16, (H + 15) // 16 * 16)
    padl = R & 7
    zpitch = (W + padl + 7) // 8 * 8
    assert zpitch % 8 == 0 and zpitch >= W + padl
    ch = h_cols(split)
    Klh = ch - 16 + 32 * nks
    for bx in (0, (W + ch - 1) // ch - 1):
        x0 = bx * ch
        zc0 = x0 - R + padl
        assert zc0 % 8 == 0
        for v in range(Klh // 8):
            zc = zc0 + 8 * v
            if zc + 8 > padl and zc < padl + W:
                assert 0 <= zc and zc + 8 <= zpitch
    # vertical stores: last pixel of the last tile
    assert (H - 1) * zpitch + padl + W - 1 < H * zpitch
    # every LDS fragment read of the last row/column blocks
    Kl = rows - 16 + 32 * nks
    assert 16 * (rows // 16 - 1) + 8 * 3 + 32 * (nks - 1) + 8 <= Kl
    assert 16 * (ch // 16 - 1) + 8 * 3 + 32 * (nks - 1) + 8 <= Klh


def test_radius_limit():
    assert shape(False, 120, 500) is not None and shape(True, 120, 500) is not None
    assert shape(False, 121, 500) is None and shape(True, 121, 500) is None


def xcd_tile(i, per):
    return (i % 8) * per + i // 8


@pytest.mark.parametrize("n", [1, 7, 8, 9, 128, 1000, 8193])
def test_xcd_tile_map_is_a_bijection(n):
    """Launch index -> tile: every tile exactly once, extra indices out of range."""
    per = (n + 7) // 8
    tiles = [xcd_tile(i, per) for i in range(8 * per)]
    assert sorted(t for t in tiles if t < n) == list(range(n))


def group_find(start, n, bid):
    lo, hi = 0, n - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if start[mid] <= bid:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("blocks", [[1], [3, 0, 5], [0, 0, 4, 0], [7, 1, 1, 9, 2], [0, 8, 0, 0, 8]])
def test_grouped_launch_block_map(blocks):
    """Blocks of a grouped launch -> (image, local block), as the grouped
    kernels decompose them: every local block of every image exactly once,
    images without blocks skipped."""
    start = np.concatenate([[0], np.cumsum(blocks)]).astype(int)
    n = len(blocks)
    seen = []
    for bid in range(start[-1]):
        i = group_find(start, n, bid)
        assert start[i] <= bid < start[i + 1]
        seen.append((i, bid - start[i]))
    assert seen == [(i, l) for i in range(n) for l in range(blocks[i])]


@pytest.mark.parametrize("gx,gy,gz", [(1, 1, 1), (8, 3, 1), (5, 7, 2)])
def test_group_grid_decomposition(gx, gy, gz):
    got = [(l % gx, (l // gx) % gy, l // (gx * gy)) for l in range(gx * gy * gz)]
    assert sorted(got) == [(x, y, z) for x in range(gx) for y in range(gy) for z in range(gz)]


@pytest.mark.parametrize("nvec", [1, 15, 16, 17, 22, 30, 32, 33, 46, 64])
def test_horizontal_staging_lane_map(nvec):
    """Each wave stages 16 of the 64 LDS rows; Lr lanes (16, 32 or 64, the
    smallest >= nvec) take one row, so an instruction covers 64 / Lr rows:
    every (row, vector < nvec) is written exactly once, by lanes that exist."""
    lrs = 4 if nvec <= 16 else (5 if nvec <= 32 else 6)
    rpi = 64 >> lrs
    ninst = 16 >> (6 - lrs)
    seen = []
    for wv in range(4):
        for j in range(ninst):
            for lane in range(64):
                vl, sub = lane & ((1 << lrs) - 1), lane >> lrs
                if vl >= nvec:
                    continue
                rr = wv + 4 * (j * rpi + sub)
                seen.append((rr, vl))
    assert sorted(seen) == [(rr, v) for rr in range(64) for v in range(nvec)]
