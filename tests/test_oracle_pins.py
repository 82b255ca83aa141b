"""Pins of the FP64 oracle to facts the paper and mathematics fix.

None of these compare the oracle with itself: each side is a printed value of
the paper (tests/golden), a closed form, exact rational arithmetic, a brute
force, an independent library routine, or an invariant of the method.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as o
from bfsynth import config_image, gen_random, CONFIGS


def _golden(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as fh:
        return json.load(fh)


# ----------------------------------------------------------- Table 1 / Fig. 1
def test_table1_order(golden_dir):
    g = _golden(golden_dir, "table1_order.json")
    got = [o.order(g["T"], s) for s in g["sigma_r"]]
    assert got == g["N0"]


def test_fig1_truncation(golden_dir):
    g = _golden(golden_dir, "fig1_truncation.json")
    N = o.order(g["T"], g["sigma_r"])
    assert N == g["N"]
    M = o.trunc_exact(N, g["eps"])
    assert M == g["M"] == o.exact_trunc(N, g["eps"])
    kept = N - 2 * M + 1
    assert kept == g["kept"] and 2 * M == g["dropped"]
    assert round(100.0 * 2 * M / (N + 1)) == g["dropped_percent_approx"]
    # the dropped mass is within eps, the kept mass above 1 - eps (exact)
    dropped = 2 * o.exact_cum(N, M - 1)
    assert dropped <= Fraction(g["eps"])


def test_fig9_jump(golden_dir):
    g = _golden(golden_dir, "fig9_jump.json")
    lo = o.order(g["T"], g["sigma_r_below"])
    hi = o.order(g["T"], g["sigma_r_above"])
    L_lo = lo - 2 * o.trunc_rule(lo, g["sigma_r_below"], g["eps"])
    L_hi = hi - 2 * o.trunc_rule(hi, g["sigma_r_above"], g["eps"])
    assert lo < 1.15 * hi
    assert L_lo > 1.5 * L_hi


def test_table3_recorded_but_unpinned(golden_dir):
    g = _golden(golden_dir, "table3_unpinned.json")
    got = [o.order(255, s) for s in g["sigma_r"]]
    # Table 1 and Table 3 disagree with each other for these sigma_r
    assert got != g["N0_before_printed"]


# ------------------------------------------------------- order and truncation
@pytest.mark.parametrize("eps", [0.05, 0.03, 1e-2, 1e-3, 1e-4])
def test_trunc_exact_matches_rationals(eps):
    for N in list(range(1, 120)) + [150, 199, 263, 300, 411]:
        assert o.trunc_exact(N, eps) == o.exact_trunc(N, eps), N


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4])
def test_chernoff_rule_is_conservative(eps):
    # eq. (Chernoff) must never drop more than eps/2 per side (exact check),
    # and never keep fewer terms than the exact rule
    for N in [1, 2, 5, 17, 64, 101, 263, 500, 1053, 2718]:
        M = o.trunc_chernoff(N, eps)
        assert 0 <= M <= N // 2
        if M > 0:
            assert o.exact_cum(N, M - 1) <= Fraction(eps) / 2
        if N <= 1100:
            assert M <= o.exact_trunc(N, eps)


@pytest.mark.parametrize("eps", [0.05, 1e-2, 1e-3, 1e-4, 1e-6])
def test_chernoff_rule_sets_the_bound_to_half_eps(eps):
    """Eq. (Chernoff) comes from setting the Chernoff bound
    exp(-(N - 2M)^2 / (4N)) of the binomial tail equal to eps/2 (Section 3):
    M is the largest non-negative integer whose bound is <= eps/2, so the
    bound at M holds and the bound at M + 1 would fail.  A natural log, the
    eps/2 budget and rounding down are each fixed by this; log(1/eps),
    log10, or rounding up fail it for some N of the sweep."""
    def bound(N, M):
        return math.exp(-((N - 2 * M) ** 2) / (4.0 * N))
    for N in list(range(1, 400)) + [411, 500, 1053, 1582, 2718, 2929, 5000]:
        M = o.trunc_chernoff(N, eps)
        assert 0 <= M <= N // 2
        if M > 0:
            assert bound(N, M) <= eps / 2, (N, M)
        else:  # M = 0 is the clamp when even M = 0 misses the bound, or the largest fit
            assert bound(N, 0) <= eps / 2 or 2 * math.sqrt(N * math.log(2 / eps)) >= N
        if N - 2 * (M + 1) >= 0:
            assert bound(N, M + 1) > eps / 2, (N, M)


def test_chernoff_rule_worked_values():
    """Worked values of eq. (Chernoff) at the Fig. 1 setting, from the closed
    form by hand: N = 263, eps = 0.01 gives (263 - sqrt(4 263 ln 200))/2
    = (263 - 74.67...)/2 = 94.16..., so M = 94 and N - 2M + 1 = 76 kept terms
    (the exact rule keeps 42: the estimate is conservative)."""
    v = 0.5 * (263 - math.sqrt(4 * 263 * math.log(200.0)))
    assert 94.0 < v < 94.5
    assert o.trunc_chernoff(263, 0.01) == 94
    assert o.trunc_exact(263, 0.01) == 111


def test_band_rule_selects_per_sigma_r():
    N = 263
    assert o.trunc_rule(N, 41.0, 1e-3) == 0
    assert o.trunc_rule(N, 20.0, 1e-3) == o.exact_trunc(N, 1e-3)
    assert o.trunc_rule(N, 10.0, 1e-3) == o.trunc_chernoff(N, 1e-3)


# --------------------------------------------------------------- eq. (expansion)
@pytest.mark.parametrize("N", [1, 2, 7, 29, 66, 263, 1053, 2718])
def test_binomial_expansion_identity(N):
    sr = 10.0
    T = sr * math.sqrt(N / 0.405)
    for s in np.linspace(-T, T, 41):
        lhs = math.cos(s / (math.sqrt(N) * sr)) ** N
        rhs = o.phi_eps(s, N, 0, sr)
        assert abs(lhs - rhs) < 1e-12 * max(1.0, N / 100.0), (N, s)


def test_coefficient_facts():
    for N in [4, 10, 64, 263, 1000]:
        c = np.array([o.coef(N, n) for n in range(N + 1)])
        assert abs(c.sum() - 1.0) < 1e-12
        assert np.all(c > 0)
        k = int(np.argmax(c))
        assert np.all(np.diff(c[:k + 1]) >= 0) and np.all(np.diff(c[k:]) <= 0)
        assert abs(c[0] - 2.0 ** -N) <= 1e-12 * 2.0 ** -N
        assert abs(c[0] - c[N]) <= 1e-12 * c[0]
        # Stirling: largest ~ sqrt(2/(pi N)).  The ratio smallest/largest is then
        # 2^-N sqrt(pi N / 2); the closed form printed next to these two facts,
        # (pi N 2^(2N-1))^(-1/2), differs from it by the factor 2/(pi N) and is
        # not used (the two stated facts agree with each other and with c).
        assert abs(c.max() / math.sqrt(2.0 / (math.pi * N)) - 1.0) < 1.0 / N
        log_ratio = math.log(c[0]) - math.log(c.max())
        pred = -N * math.log(2.0) + 0.5 * math.log(math.pi * N / 2.0)
        assert abs(log_ratio - pred) < 1.0 / N


@pytest.mark.parametrize("sr,eps", [(5.0, 0.03), (10.0, 1e-2), (20.0, 1e-3), (30.0, 1e-3)])
def test_truncation_error_bound(sr, eps):
    T = 255.0
    N = o.order(T, sr)
    M = o.trunc_rule(N, sr, eps)
    dropped = 2 * sum(o.coef(N, n) for n in range(M))
    assert dropped <= eps
    worst = 0.0
    low = 1.0
    for s in np.linspace(-T, T, 801):
        a, b = o.phi(s, N, sr), o.phi_eps(s, N, M, sr)
        worst = max(worst, abs(a - b))
        low = min(low, b)
    assert worst <= dropped + 1e-12
    assert low >= -eps - 1e-12


def test_raised_cosine_converges_to_gaussian():
    sr = 10.0
    errs = []
    for N in [10, 30, 100, 300, 1000]:
        T = sr * math.sqrt(N / 0.405)
        s = np.linspace(-T, T, 2001)
        err = np.abs(np.cos(s / (math.sqrt(N) * sr)) ** N - np.exp(-s * s / (2 * sr * sr))).max()
        errs.append(err)
        assert err * N < 1.0  # O(1/N)
        assert abs(o.phi(s[7], N, sr) - math.cos(s[7] / (math.sqrt(N) * sr)) ** N) < 1e-14
    assert all(a > b for a, b in zip(errs, errs[1:]))


# ------------------------------------------------------ Algorithm 1 / Appendix
@pytest.mark.parametrize("n", [1, 2, 5, 17, 100, 257])
@pytest.mark.parametrize("R", [0, 1, 3, 10, 50])
def test_maxfilter_equals_bruteforce(n, R):
    rng = np.random.default_rng(n * 1000 + R)
    x = rng.integers(0, 256, n).astype(float)
    ref = np.array([x[max(0, i - R):min(n, i + R + 1)].max() for i in range(n)])
    assert np.array_equal(o.maxfilter_1d(x, R), ref)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (7, 5), (16, 16), (31, 23)])
@pytest.mark.parametrize("R", [0, 1, 2, 5, 20])
def test_range_T_equals_bruteforce(shape, R):
    f = gen_random(11 + shape[0] * 7 + R, *shape, dtype="u8").astype(float)
    T = o.range_T(f, R)
    mx, mn = o.brute_window_extrema(f, R)
    T_plus = (f - mn).max()
    T_minus = (mx - f).max()
    assert T_plus == T_minus  # Prop. 2.1
    assert T == o.brute_T(f, R) == T_minus


def test_range_T_float_image():
    f = gen_random(5, 40, 33, dtype="f32").astype(float)
    for R in (1, 4, 9):
        assert o.range_T(f, R) == o.brute_T(f, R)


# ---------------------------------------------------------- spatial operators
def test_fir_operator_matches_scipy():
    from scipy.ndimage import correlate1d
    rng = np.random.default_rng(3)
    for n, sigma, R in [(1, 1.0, 3), (13, 2.0, 6), (100, 3.0, 9), (64, 10.0, 30)]:
        x = rng.normal(size=n)
        j = np.arange(-R, R + 1)
        w = np.exp(-j * j / (2 * sigma * sigma))
        ref = correlate1d(x, w, mode="constant", cval=0.0)
        assert np.allclose(o.blur_1d(x, "fir", sigma, R), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("sigma", [0.6, 1.0, 2.0, 3.0, 8.0, 10.0, 16.0])
def test_iir_operator_matches_lfilter(sigma):
    from scipy.signal import lfilter
    c = o.yvv_coefs(sigma)
    B, a1, a2, a3 = c
    rng = np.random.default_rng(int(sigma * 10))
    for n in (1, 7, 50, 300):
        x = rng.normal(size=n)
        pad = int(60 * sigma) + 200
        xp = np.concatenate([x, np.zeros(pad)])
        w = lfilter([B], [1.0, -a1, -a2, -a3], xp)
        y = lfilter([B], [1.0, -a1, -a2, -a3], w[::-1])[::-1]
        assert np.allclose(o.blur_1d(x, "iir", sigma), y[:n], rtol=0, atol=1e-12)


@pytest.mark.parametrize("sigma,tol", [(1.0, 0.10), (2.0, 0.06), (3.0, 0.045), (8.0, 0.03),
                                       (10.0, 0.025), (16.0, 0.02), (30.0, 0.015)])
def test_iir_impulse_response_is_gaussian(sigma, tol):
    """The Young-van Vliet design approximates the sampled Gaussian: unit mass,
    positive, even, within a few percent of the peak."""
    n = int(80 * sigma) + 101
    e = np.zeros(n)
    mid = n // 2
    e[mid] = 1.0
    h = o.blur_1d(e, "iir", sigma)
    t = np.arange(n) - mid
    g = np.exp(-t * t / (2 * sigma * sigma))
    g /= g.sum()
    assert abs(h.sum() - 1.0) < 1e-9
    assert h.min() > -1e-6 * h.max()  # tiny negative tail at large sigma
    assert np.allclose(h[mid - 40:mid + 41], h[mid - 40:mid + 41][::-1], atol=1e-14)
    assert np.abs(h - g).max() < tol * g.max()
    var = (t * t * h).sum()
    assert 0.95 * sigma ** 2 < var < 1.6 * sigma ** 2


@pytest.mark.parametrize("n,R", [(1, 0), (1, 3), (9, 2), (40, 5), (300, 20), (17, 40)])
def test_box_operator_pins(n, R):
    """The constant spatial filter of radius R (Section 4): the count of the
    clipped window on a constant line, the difference of cumulative sums,
    scipy's uniform filter times the window size, and the banded all-ones
    matrix."""
    from scipy.ndimage import uniform_filter1d
    i = np.arange(n)
    cnt = np.minimum(i + R, n - 1) - np.maximum(i - R, 0) + 1
    assert np.array_equal(o.blur_1d(np.ones(n), "box", 1.0, R), cnt.astype(float))
    rng = np.random.default_rng(n * 7 + R)
    x = rng.normal(size=n)
    c = np.concatenate([[0.0], np.cumsum(x)])
    ref = c[np.minimum(i + R, n - 1) + 1] - c[np.maximum(i - R, 0)]
    assert np.allclose(o.blur_1d(x, "box", 1.0, R), ref, rtol=0, atol=1e-11)
    if 2 * R + 1 <= n:
        uf = uniform_filter1d(x, 2 * R + 1, mode="constant", cval=0.0) * (2 * R + 1)
        assert np.allclose(o.blur_1d(x, "box", 1.0, R), uf, rtol=0, atol=1e-11)
    S = o.operator_matrix(n, "box", 1.0, R)
    assert np.array_equal(S, (np.abs(i[:, None] - i[None, :]) <= R).astype(float))


def test_operators_are_symmetric_matrices():
    for op, s, R in (("fir", 2.0, 6), ("iir", 2.0, 0), ("iir", 5.0, 0), ("box", 1.0, 3)):
        S = o.operator_matrix(23, op, s, R)
        assert np.allclose(S, S.T, atol=1e-13)


# ------------------------------------------------------- the filter itself
TINY = [(1, 1, "mixed"), (1, 7, "mixed"), (7, 1, "mixed"), (7, 5, "noise"), (12, 12, "mixed"),
        (9, 11, "step"), (6, 6, "const")]


@pytest.mark.parametrize("H,W,kind", TINY)
@pytest.mark.parametrize("op", ["fir", "iir", "box"])
def test_shiftable_equals_direct(H, W, kind, op):
    """The expansion of eqs. (f1)/(f2) reproduces eq. (BF) with the same
    truncated range kernel and the same spatial operator."""
    f = gen_random(100 + H * 13 + W, H, W, "u8", kind).astype(float)
    ss, R, sr, eps = 1.5, 4, 25.0, 1e-3
    T = o.range_T(f, R)
    N = o.order(T, sr)
    M = o.trunc_rule(N, sr, eps)
    out, P, Q, bad = o.shiftable_bf(f, op, ss, R, N, M, sr)
    Sv = o.operator_matrix(H, op, ss, R)
    Sh = o.operator_matrix(W, op, ss, R)
    ref = o.direct_bf_dense(f, Sv, Sh, o.phi_eps_vec(N, M, sr))
    assert bad == 0
    assert np.allclose(out, ref, rtol=1e-9, atol=1e-9 * 255)


def qneg_image(H=100, W=131, bg=200.0, spot=60.0):
    """Background `bg` with isolated pixels of value `spot` every 32 rows and
    33 columns: at sigma_r = 25, eps = 0.05 and T = 255 the truncated kernel
    phi_eps (eq. (approx)) dips to about -0.021 at the difference 140, so the
    denominator (f2) of each isolated pixel is its own weight phi_eps(0) ~ 1
    minus about 0.021 times the rest of the spatial mass: negative for
    sigma_s >= 3 (Section 3 allows overshoots down to -eps)."""
    f = np.full((H, W), bg)
    ys, xs = np.meshgrid(np.arange(10, H, 32), np.arange(12, W, 33), indexing="ij")
    f[ys, xs] = spot
    return f, ys.ravel(), xs.ravel()


@pytest.mark.parametrize("op", ["fir", "iir", "box"])
def test_nonpositive_denominator_fallback(op):
    """Where the denominator (f2) is not positive the output is the input pixel
    and the pixel is counted.  The pixels so counted are exactly those where
    eq. (BF) evaluated directly (materialised operator, same phi_eps) has a
    non-positive denominator, on a crop small enough for the dense form."""
    sr, eps, ss = 25.0, 0.05, 4.0
    R = 12
    N = o.order(255.0, sr)
    M = o.trunc_rule(N, sr, eps)
    assert (N, M) == (42, 15)
    k = o.phi_eps_vec(N, M, sr)
    assert k(np.array([140.0]))[0] < -0.02
    f, ys, xs = qneg_image(30, 58)
    out, P, Q, bad = o.shiftable_bf(f, op, ss, R, N, M, sr)
    H, W = f.shape
    Sv = o.operator_matrix(H, op, ss, R)
    Sh = o.operator_matrix(W, op, ss, R)
    Wsp = np.einsum("ac,bd->abcd", Sv, Sh).reshape(H * W, H * W)
    fv = f.ravel()
    den = (Wsp * k(fv[None, :] - fv[:, None])).sum(axis=1).reshape(H, W)
    num = (Wsp * k(fv[None, :] - fv[:, None]) @ fv).reshape(H, W)
    assert np.allclose(Q, den, rtol=1e-9, atol=1e-9 * np.abs(den).max())
    neg = den <= 0
    assert neg.sum() == bad == len(ys) == 2
    assert np.all(neg[ys, xs])
    assert np.array_equal(out[neg], f[neg])
    assert np.allclose(out[~neg], num[~neg] / den[~neg], rtol=1e-9, atol=1e-9)
    # the full-size image the GPU tests use: one count per isolated pixel
    f2, ys2, xs2 = qneg_image()
    r = o.algorithm2(f2, op, 6.0, 18, sr, eps, 255.0, False, 255.0)
    assert r["n_nonpos"] == len(ys2) == 12
    assert np.array_equal(r["out"][ys2, xs2], f2[ys2, xs2])


@pytest.mark.parametrize("op", ["fir", "iir", "box"])
def test_constant_image_unchanged(op):
    for v in (0.0, 17.0, 255.0):
        f = np.full((20, 17), v)
        r = o.algorithm2(f, op, 2.0, 6, 10.0, 1e-3, 255.0, True)
        assert r["T"] == 0 and r["N"] == 1
        assert np.allclose(r["out"], v, atol=1e-9)


@pytest.mark.parametrize("op", ["fir", "iir", "box"])
def test_affine_and_reflection_invariance(op):
    f = gen_random(7, 24, 20, "u8").astype(float)
    ss, R, sr, eps = 2.0, 6, 15.0, 1e-3
    base = o.algorithm2(f, op, ss, R, sr, eps, 255.0, True)
    # f -> 257 f (8-bit to 16-bit), sigma_r and range scale too
    big = o.algorithm2(257.0 * f, op, ss, R, 257.0 * sr, eps, 65535.0, True)
    assert big["N"] == base["N"] and big["M"] == base["M"]
    assert np.allclose(big["out"], 257.0 * base["out"], rtol=0, atol=1e-8 * 65535)
    # f -> f + b
    sh = o.algorithm2(f + 40.0, op, ss, R, sr, eps, 255.0, True)
    assert np.allclose(sh["out"], base["out"] + 40.0, atol=1e-8 * 255)
    # f -> 255 - f
    ref = o.algorithm2(255.0 - f, op, ss, R, sr, eps, 255.0, True)
    assert np.allclose(ref["out"], 255.0 - base["out"], atol=1e-8 * 255)


@pytest.mark.parametrize("op", ["fir", "iir", "box"])
def test_transpose_commutes(op):
    f = gen_random(9, 19, 26, "u8").astype(float)
    a = o.algorithm2(f, op, 2.5, 8, 20.0, 1e-3, 255.0, True)
    b = o.algorithm2(f.T.copy(), op, 2.5, 8, 20.0, 1e-3, 255.0, True)
    assert np.allclose(a["out"].T, b["out"], atol=1e-9)


def test_box_direct_matches_expansion():
    """Eq. (BF) evaluated directly with the box filter at sampled pixels equals
    the expansion (Algorithm 2 with the box operator), at the paper's box
    setting (radius 20, sigma_r = 5, eps = 0.01) on a synthetic image."""
    f = gen_random(21, 90, 110, "u8").astype(float)
    r = o.algorithm2(f, "box", 1.0, 20, 5.0, 1e-2, 255.0, True)
    rng = np.random.default_rng(5)
    ys = np.concatenate([rng.integers(0, 90, 60), [0, 89, 0, 89]])
    xs = np.concatenate([rng.integers(0, 110, 60), [0, 109, 109, 0]])
    d = o.direct_box_at(f, 20, r["N"], r["M"], 5.0, ys, xs)
    assert np.allclose(r["out"][ys, xs], d, rtol=0, atol=1e-9 * 255)


def test_error_to_gaussian_bf_shrinks():
    """As eps -> 0 and the order grows the result approaches the Gaussian BF
    with the same spatial operator (Section 1.3, eq. (RCconv))."""
    f = gen_random(21, 14, 14, "u8", "mixed").astype(float)
    ss, R, sr = 2.0, 6, 30.0
    Sv = o.operator_matrix(14, "fir", ss, R)
    gauss = o.direct_bf_dense(f, Sv, Sv, lambda s: np.exp(-s * s / (2 * sr * sr)))
    errs = []
    for tv in (255.0, 1020.0, 4080.0):
        N = o.order(tv, sr)
        out, _, _, _ = o.shiftable_bf(f, "fir", ss, R, N, 0, sr)
        errs.append(np.abs(out - gauss).max())
    assert errs[0] > errs[1] > errs[2]
    e_eps = []
    N = o.order(1020.0, sr)
    for eps in (1e-1, 1e-2, 1e-4):
        M = o.trunc_exact(N, eps)
        out, _, _, _ = o.shiftable_bf(f, "fir", ss, R, N, M, sr)
        e_eps.append(np.abs(out - gauss).max())
    assert e_eps[0] > e_eps[1] > e_eps[2]


def test_workload1_crop_crosscheck():
    """Workload 1: the expansion equals eq. (BF) evaluated directly on the
    central 64x64 crop with the full-image neighbourhood (FIR operator)."""
    c = CONFIGS[1]
    f = config_image(1).astype(float)
    r = o.algorithm2(f, "fir", c["sigma_s"], c["radius"], c["sigma_r"], c["eps"], 255.0, False,
                     c["t_value"])
    assert (r["N"], r["M"]) == (29, 6)
    ys, xs = np.mgrid[96:160, 96:160]
    d = o.direct_fir_at(f, c["sigma_s"], c["radius"], r["N"], r["M"], c["sigma_r"],
                        ys.ravel(), xs.ravel())
    assert np.allclose(r["out"][96:160, 96:160].ravel(), d, rtol=0, atol=1e-9)
