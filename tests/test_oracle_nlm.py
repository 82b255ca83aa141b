"""Pins of the non-local-means oracle (eqs. (NL1), (NL2) of the paper's
closing section): the multi-index expansion against the direct sums, p = 1
against the bilateral filter, the product identity of the expanded kernels,
the bound |s_k| <= T of Algorithm 1, the pair count, invariances, and the
limit of the Gaussian non-local means."""
import math

import numpy as np
import pytest

import oracle as o
from oracle import nlm
from bfsynth import gen_random

OFF3 = [(0, 0), (0, 1), (1, 0)]
OFF4 = [(0, 0), (0, -1), (-1, 0), (1, 1)]


@pytest.mark.parametrize("op", ["box", "fir"])
@pytest.mark.parametrize("offsets", [OFF3, [(0, 0), (2, -1)]])
def test_shiftable_equals_direct(op, offsets):
    """The expansion the GPU runs (one term per folded multi-index) equals
    eqs. (NL1)/(NL2) evaluated directly with the product of truncated kernels."""
    f = gen_random(7, 9, 11, "u8", "mixed").astype(np.float64)
    N, M, sr = 7, 1, 60.0
    a = nlm.nlm_direct(f, offsets, op, 1.5, 3, N, M, sr)
    b = nlm.nlm_shiftable(f, offsets, op, 1.5, 3, N, M, sr)
    assert a[3] == b[3] == 0
    assert np.abs(a[0] - b[0]).max() < 1e-9
    assert np.abs(a[2] - b[2]).max() < 1e-9 * np.abs(a[2]).max()


def test_one_sample_patch_is_the_bilateral_filter():
    """With p = 1 (u_1 = 0) eqs. (NL1)/(NL2) are eq. (BF) with the window
    operator: the FIR and box bilateral filters of the oracle."""
    f = gen_random(9, 23, 29, "u8", "mixed").astype(np.float64)
    ss, R, sr, eps = 2.0, 6, 25.0, 1e-3
    N = o.order(255, sr)
    M = o.trunc_rule(N, sr, eps)
    out, _, _, _ = nlm.nlm_direct(f, [(0, 0)], "fir", ss, R, N, M, sr)
    ref = o.algorithm2(f, "fir", ss, R, sr, eps, 255.0, False, 255.0)
    assert (ref["N"], ref["M"]) == (N, M)
    assert np.abs(out - ref["out"]).max() < 1e-9
    ys, xs = np.array([0, 22, 11, 3]), np.array([0, 28, 14, 20])
    outb, _, _, _ = nlm.nlm_direct(f, [(0, 0)], "box", 1.0, R, N, M, sr)
    assert np.abs(outb[ys, xs] - o.direct_box_at(f, R, N, M, sr, ys, xs)).max() < 1e-9


@pytest.mark.parametrize("N,M,p", [(7, 0, 3), (16, 2, 3), (29, 6, 2), (12, 3, 4)])
def test_product_identity_and_pair_count(N, M, p):
    """prod_k phi_eps(s_k) = sum over folded multi-indices of
    C_m cos(alpha sum_k m_k s_k) (cos of a sum of angles, conjugate pairs
    folded), for random s; and the fold leaves (L^p + z)/2 terms."""
    sr = 20.0
    rng = np.random.default_rng(N * 100 + p)
    S = rng.uniform(-255, 255, (50, p))
    alpha = 1.0 / (math.sqrt(N) * sr)
    terms = nlm.multi_indices(N, M, p)
    assert len(terms) == nlm.pair_count(N, M, p)
    mv = np.array([t[0] for t in terms], dtype=np.float64)
    cw = np.array([t[1] for t in terms])
    lhs = np.prod([[o.phi_eps(float(s), N, M, sr) for s in row] for row in S], axis=1)
    rhs = (cw[None, :] * np.cos(alpha * S @ mv.T)).sum(1)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_every_patch_difference_is_within_T():
    """|s_k| = |f(x + u_k) - f(x - y + u_k)| <= T of Algorithm 1 for every x,
    |y| <= R and k, with clamped patch samples (brute force)."""
    f = gen_random(2, 30, 26, "u8", "noise").astype(np.float64)
    R = 3
    T = o.range_T(f, R)
    P = nlm.patch_stack(f, OFF4)
    H, W = f.shape
    worst = 0.0
    for y in range(H):
        for x in range(W):
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if 0 <= y - dy < H and 0 <= x - dx < W:
                        worst = max(worst, np.abs(P[:, y, x] - P[:, y - dy, x - dx]).max())
    assert worst <= T
    assert worst == T  # the centre sample (u_1 = 0) attains it


def test_constant_reflection_transpose():
    f = gen_random(4, 17, 19, "u8", "mixed").astype(np.float64)
    N, M, sr = 16, 2, 40.0
    c, _, _, _ = nlm.nlm_direct(np.full((9, 8), 123.0), OFF3, "box", 1.0, 2, N, M, sr)
    assert np.abs(c - 123.0).max() < 1e-9
    a = nlm.nlm_direct(f, OFF3, "box", 1.0, 3, N, M, sr)[0]
    b = nlm.nlm_direct(255.0 - f, OFF3, "box", 1.0, 3, N, M, sr)[0]
    assert np.abs((255.0 - b) - a).max() < 1e-9
    t = nlm.nlm_direct(f.T.copy(), [(dx, dy) for dy, dx in OFF3], "box", 1.0, 3, N, M, sr)[0]
    assert np.abs(t.T - a).max() < 1e-9


def test_tends_to_gaussian_nlm():
    """As eps -> 0 and N grows (T raised, eq. (RCconv)) the filter tends to
    the non-local means with the Gaussian product kernel."""
    f = gen_random(6, 14, 15, "u8", "mixed").astype(np.float64)
    sr, R = 40.0, 2
    P = nlm.patch_stack(f, OFF3)
    H, W = f.shape
    gauss = np.empty_like(f)
    for y in range(H):
        for x in range(W):
            num = den = 0.0
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    if 0 <= y - dy < H and 0 <= x - dx < W:
                        s = P[:, y, x] - P[:, y - dy, x - dx]
                        k = math.exp(-(s * s).sum() / (2 * sr * sr))
                        num += k * f[y - dy, x - dx]
                        den += k
            gauss[y, x] = num / den
    errs = []
    for T in (255, 510, 1020):
        N = o.order(T, sr)
        errs.append(np.abs(nlm.nlm_direct(f, OFF3, "box", 1.0, R, N, 0, sr, smax=255)[0] - gauss).max())
    assert errs[0] > errs[1] > errs[2]
