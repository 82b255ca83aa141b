"""Pins of the polynomial-kernel oracle (eqs. (RP), (RPconv), Section 1.3) to
facts the paper and mathematics fix: the positivity threshold N0, the limit
of eq. (RPconv), the shiftable identity written out in exact rational
arithmetic, the uniform truncation bound, SHIFTABLE-BF against eq. (BF)
evaluated by brute force, and the invariances of the filter."""
import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle as o
from oracle import poly as rp
from bfsynth import gen_random

L8 = 255.0


@pytest.mark.parametrize("T,sr", [(255, 30), (255, 10), (255, 60), (100, 7), (255, 200), (40, 3.3)])
def test_order_is_the_smallest_positive_monotone_one(T, sr):
    """N >= N0 = 0.5 (T/sr)^2 makes the base 1 - s^2/(2 N sr^2) non-negative
    on [-T, T] (Section 1.3); one order less makes it negative at s = T, so
    that phi is no longer monotone there (unless N = 1 already)."""
    N = rp.rp_order(T, sr)
    assert N >= 0.5 * (T / sr) ** 2 and N >= 1
    s = np.linspace(0.0, T, 2001)
    base = 1.0 - s * s / (2.0 * N * sr * sr)
    assert base.min() >= -1e-15
    phi = rp.rp_kernel(s, N, sr)
    assert np.all(np.diff(phi) <= 1e-15) and phi[0] == 1.0
    if N > 1:
        assert 1.0 - T * T / (2.0 * (N - 1) * sr * sr) < 0


def test_rpconv_limit():
    """eq. (RPconv): max_{|s|<=T} |phi_N(s) - exp(-s^2/2 sr^2)| falls to 0 as N
    grows, at the rate 1/N (the first term of log(1-u)N = -uN - u^2 N/2 ...)."""
    T, sr = 255.0, 30.0
    s = np.linspace(-T, T, 4001)
    g = np.exp(-s * s / (2 * sr * sr))
    errs = []
    Ns = [rp.rp_order(T, sr) * k for k in (1, 2, 4, 8, 16, 32)]
    for N in Ns:
        errs.append(np.abs(rp.rp_kernel(s, N, sr) - g).max())
    assert all(b < a for a, b in zip(errs, errs[1:]))
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(1.7 < r < 2.3 for r in ratios[2:])  # O(1/N)


def _exact_phi(a, b, N, sr2N):
    """(1 - (a-b)^2 / sr2N)^N in rationals."""
    u = Fraction(a - b) ** 2 / sr2N
    return (1 - u) ** N


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_shiftable_identity_exact_rationals(N):
    """Shiftability (Section 1.2): phi(a - b) = sum_i c_i(b) phi_i(a) with the
    monomial basis phi_i(a) = a^i and coefficients from the binomial theorem,
    c_i(b) = sum_k C(N,k) (-1/K)^k C(2k,i) (-b)^(2k-i), K = 2 N sr^2 -- checked
    in exact rationals against the closed form; the Chebyshev coefficients of
    the oracle reproduce the same polynomial in a."""
    sr = Fraction(7, 2)
    K = 2 * N * sr * sr
    for b in (0, 3, 11, 20):
        coef = [Fraction(0)] * (2 * N + 1)
        for k in range(N + 1):
            for i in range(2 * k + 1):
                coef[i] += math.comb(N, k) * (Fraction(-1) / K) ** k * math.comb(2 * k, i) * Fraction(-b) ** (2 * k - i)
        for a in range(0, 21, 4):
            lhs = _exact_phi(a, b, N, K)
            rhs = sum(c * Fraction(a) ** i for i, c in enumerate(coef))
            assert lhs == rhs
        # the oracle's Chebyshev form on [0, L] represents the same polynomial
        L = 20.0
        C = rp.rp_coefs(N, float(sr), L, [b])[0]
        mono = npcheb.cheb2poly(C)  # in x = (a - L/2)/(L/2)
        a = np.linspace(0, L, 9)
        got = np.polynomial.polynomial.polyval(rp.to_unit(a, L), mono)
        want = np.array([float(sum(c * Fraction(float(v)) ** i for i, c in enumerate(coef))) for v in a])
        assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("sr", [30.0, 15.0, 10.0, 5.0])
def test_chebyshev_expansion_equals_kernel(sr):
    """Untruncated: sum_{j<=2N} c_j(b) T_j(x(a)) = phi_N(a - b) for all integer
    a, b in [0, 255], to 1e-9 (the kernel's peak is 1); coefficients above
    degree 2N vanish (interpolating at more points adds only zeros)."""
    N = rp.rp_order(L8, sr)
    vals = np.arange(256.0)
    C = rp.rp_coefs(N, sr, L8, vals)
    a = vals[:, None] * np.ones((1, 256))
    b = np.ones((256, 1)) * vals[None, :]
    got = rp.rp_kernel_trunc(a, b, C, vals, L8)
    assert np.abs(got - rp.rp_kernel(a - b, N, sr)).max() < 1e-9  # FP64 rounding over 2N+1 <= 2603 terms
    hi = npcheb.chebinterpolate(lambda x: rp.rp_kernel(127.5 * (x + 1) - 40.0, N, sr), 2 * N + 6)
    assert np.abs(hi[2 * N + 1:]).max() < 1e-12


@pytest.mark.parametrize("sr,eps", [(30.0, 1e-3), (10.0, 1e-3), (20.0, 1e-2), (60.0, 1e-4)])
def test_truncation_bound_and_minimality(sr, eps):
    """|phi_N(a - b) - phi_J(a, b)| <= eps for all intensities (the uniform
    bound of the rule), and J is the smallest order the rule allows."""
    tab = rp.rp_table(sr, eps, L8, L8)
    N, J = tab["N"], tab["J"]
    full = rp.rp_coefs(N, sr, L8, tab["values"])
    sup = np.abs(full).max(0)
    assert sup[J + 1:].sum() <= eps < sup[J:].sum()
    vals = tab["values"]
    a = vals[:, None] * np.ones((1, 256))
    b = np.ones((256, 1)) * vals[None, :]
    err = np.abs(rp.rp_kernel_trunc(a, b, tab["C"], vals, L8) - rp.rp_kernel(a - b, N, sr))
    assert err.max() <= eps
    assert J < 2 * N or N <= 2


def _direct_dense(f, Sv, Sh, kern):
    """Eq. (BF) by brute force: weight of y in the output at x is
    Sv[x1,y1] Sh[x2,y2] kern(f(y), f(x))."""
    H, W = f.shape
    out = np.empty_like(f)
    for y in range(H):
        for x in range(W):
            w = np.outer(Sv[y], Sh[x]) * kern(f, np.full_like(f, f[y, x]))
            out[y, x] = (w * f).sum() / w.sum()
    return out


@pytest.mark.parametrize("op", ["fir", "iir", "box"])
@pytest.mark.parametrize("trunc", [False, True])
def test_shiftable_equals_direct_bf(op, trunc):
    """SHIFTABLE-BF with the polynomial kernel = eq. (BF) evaluated by brute
    force with the same kernel and the same (materialised) spatial operator."""
    f = gen_random(5, 9, 11, "u8", "mixed").astype(np.float64)
    ss, R, sr, eps = 1.5, 3, 40.0, 1e-3
    res = rp.rp_shiftable_bf(f, op, ss, R, sr, eps, L8, trunc=trunc)
    Sv = o.operator_matrix(9, op, ss, R)
    Sh = o.operator_matrix(11, op, ss, R)
    tab = rp.rp_table(sr, eps, L8, L8)
    if trunc:
        kern = (lambda a, b: rp.rp_kernel_trunc(a, b, tab["C"], tab["values"], L8))
    else:
        kern = (lambda a, b: rp.rp_kernel(a - b, tab["N"], sr))
    ref = _direct_dense(f, Sv, Sh, kern)
    assert res["n_nonpos"] == 0
    assert np.abs(res["out"] - ref).max() < 1e-9


def test_direct_at_matches_shiftable_fir():
    f = gen_random(8, 40, 37, "u8", "mixed").astype(np.float64)
    ss, R, sr, eps = 2.0, 6, 20.0, 1e-3
    res = rp.rp_shiftable_bf(f, "fir", ss, R, sr, eps, L8)
    ys, xs = np.array([0, 39, 17, 5, 22]), np.array([0, 36, 18, 30, 2])
    got = rp.rp_direct_at(f, "fir", ss, R, sr, eps, L8, ys, xs)
    assert np.abs(got - res["out"][ys, xs]).max() < 1e-9


def test_constant_image_unchanged():
    f = np.full((13, 17), 77.0)
    res = rp.rp_shiftable_bf(f, "iir", 2.0, 6, 15.0, 1e-3, L8)
    assert np.abs(res["out"] - 77.0).max() < 1e-9


def test_reflection_and_transpose():
    """f -> 255 - f maps x -> -x, T_j(-x) = (-1)^j T_j(x) and c_j(255-b) =
    (-1)^j c_j(b), so the truncated filter commutes with the reflection; the
    separable operator with one sigma commutes with transposition."""
    f = gen_random(3, 21, 18, "u8", "mixed").astype(np.float64)
    a = rp.rp_shiftable_bf(f, "iir", 2.0, 6, 25.0, 1e-3, L8)["out"]
    b = rp.rp_shiftable_bf(L8 - f, "iir", 2.0, 6, 25.0, 1e-3, L8)["out"]
    assert np.abs((L8 - b) - a).max() < 1e-9
    c = rp.rp_shiftable_bf(f.T.copy(), "iir", 2.0, 6, 25.0, 1e-3, L8)["out"]
    assert np.abs(c.T - a).max() < 1e-9


def test_error_to_gaussian_bf_falls_with_order():
    """With eps -> 0 the filter tends to the Gaussian bilateral filter as N
    grows (global T raised, eq. (RPconv))."""
    f = gen_random(4, 12, 12, "u8", "mixed").astype(np.float64)
    ss, R, sr = 1.5, 4, 30.0
    Sv = o.operator_matrix(12, "fir", ss, R)
    gauss = o.direct_bf_dense(f, Sv, Sv, lambda s: np.exp(-s * s / (2 * sr * sr)))
    errs = []
    for T in (255.0, 382.5, 510.0):
        out = rp.rp_shiftable_bf(f, "fir", ss, R, sr, 1e-9, 2 * 255.0, T=T, trunc=False)["out"]
        errs.append(np.abs(out - gauss).max())
    assert errs[0] > errs[1] > errs[2]
