"""FP64 oracle of the bilateral filter with the polynomial range kernel.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 1.2 of the paper gives two shiftable range kernels: the raised cosine
of eq. (RC) and the polynomial of eq. (RP); Section 1.3 scales the latter so
that it tends to the Gaussian (eq. (RPconv)):

    phi_N(s) = (1 - s^2 / (2 N sigma_r^2))^N,

which is non-negative and monotone on [-T, T] once N >= N0 = 0.5 (T/sigma_r)^2.
SHIFTABLE-BF (Section 1.2, steps 1-4) then needs a fixed basis phi_i and
coefficients c_i(tau) with phi(s - tau) = sum_i c_i(tau) phi_i(s): for a
polynomial of degree 2N in s any basis of the polynomials of degree <= 2N
will do.

Readings of this module (the paper is silent on them):

* N = max(1, ceil(N0)): the smallest order the positivity condition allows.
* T is global: the value range of the image type (or a given T), as in the
  original SHIFTABLE-BF.  The shiftable identity holds for every intensity
  pair in the image, not only for those inside a window, so the basis has to
  be bounded over the whole value range [0, L]; intensities are mapped to
  x = (v - L/2) / (L/2) in [-1, 1].
* Basis: Chebyshev polynomials T_j(x), j = 0..2N (the monomials of the
  paper's polynomial expansion cancel catastrophically for the orders the
  small sigma_r need).  c_j(b) is the j-th Chebyshev coefficient of
  a -> phi_N(a - b) on [0, L].
* Truncation (the paper states no rule for eq. (RP)): keep j = 0..J with J
  the smallest order whose dropped coefficients satisfy
  sum_{j > J} max_b |c_j(b)| <= eps.  Since |T_j| <= 1 on [-1, 1] the
  truncated kernel is then within eps of phi_N everywhere on [0, L]^2, the
  same uniform bound the paper's truncation of eq. (approx) gives for the
  raised cosine (Section 3).
* The spatial operator and the handling of a non-positive denominator
  (output = input, pixel counted) are those of the raised-cosine oracle.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import chebyshev as npcheb

from . import oracle as _o


# ------------------------------------------------------------ the kernel
def rp_order(T: float, sigma_r: float) -> int:
    """Smallest integer N >= N0 = 0.5 (T/sigma_r)^2 (Section 1.3), at least 1."""
    return max(1, int(math.ceil(0.5 * (float(T) / float(sigma_r)) ** 2)))


def rp_kernel(s, N: int, sigma_r: float):
    """phi_N(s) = (1 - s^2 / (2 N sigma_r^2))^N, eq. (RPconv)."""
    s = np.asarray(s, dtype=np.float64)
    return (1.0 - s * s / (2.0 * N * sigma_r * sigma_r)) ** N


def to_unit(v, L: float):
    """Intensity v in [0, L] to x in [-1, 1]."""
    return (np.asarray(v, dtype=np.float64) - 0.5 * L) / (0.5 * L)


def rp_coefs(N: int, sigma_r: float, L: float, values) -> np.ndarray:
    """c[i, j]: Chebyshev coefficient j = 0..2N of a -> phi_N(a - values[i])
    on a in [0, L] (interpolation at 2N+1 Chebyshev points, exact for a
    polynomial of degree 2N up to rounding)."""
    values = np.asarray(values, dtype=np.float64)
    out = np.empty((values.size, 2 * N + 1))
    for i, b in enumerate(values):
        out[i] = npcheb.chebinterpolate(lambda x, b=b: rp_kernel(0.5 * L * (x + 1.0) - b, N, sigma_r), 2 * N)
    return out


def rp_truncation(C: np.ndarray, eps: float) -> int:
    """Smallest J with sum_{j > J} max_b |c_j(b)| <= eps."""
    sup = np.abs(C).max(axis=0)
    tail = 0.0
    J = C.shape[1] - 1
    # walk down from the top order while the dropped sum stays within eps
    while J > 0 and tail + sup[J] <= eps:
        tail += sup[J]
        J -= 1
    return J


def rp_table(sigma_r: float, eps: float, L: float, T: float, values=None):
    """Order, truncation and coefficients for global T over the integer
    intensities 0..L (or the given values)."""
    N = rp_order(T, sigma_r)
    vals = np.arange(int(L) + 1, dtype=np.float64) if values is None else np.asarray(values, np.float64)
    C = rp_coefs(N, sigma_r, L, vals)
    J = rp_truncation(C, eps)
    return dict(N=N, J=J, C=C[:, :J + 1], values=vals)


def rp_kernel_trunc(a, b, C: np.ndarray, values, L: float):
    """The truncated kernel sum_{j<=J} c_j(b) T_j(x(a)) for intensities a
    and table rows b (b must be one of `values`)."""
    values = np.asarray(values)
    rows = np.searchsorted(values, np.asarray(b, dtype=np.float64))
    Tj = npcheb.chebvander(to_unit(a, L), C.shape[1] - 1)
    return np.einsum("...j,...j->...", Tj, C[rows])


# --------------------------------------------------------- SHIFTABLE-BF
def rp_shiftable_bf(f, op, sigma_s: float, R: int, sigma_r: float, eps: float, L: float, T: float = 0.0,
                    trunc: bool = True):
    """SHIFTABLE-BF (Section 1.2) with the polynomial kernel: for every kept
    basis function phi_j = T_j(x(.)) the images F_j = f phi_j(f) and
    G_j = phi_j(f) are smoothed by the spatial operator `op` ("iir", "fir",
    "box") and combined with the coefficients c_j(f(x)) into eqs. (f1) and
    (f2).  Integer-valued images only (the coefficients are tabulated per
    intensity).  Returns dict(out, N, J, n_nonpos, P, Q)."""
    f = np.asarray(f, dtype=np.float64)
    if not np.array_equal(f, np.rint(f)):
        raise ValueError("integer intensities only")
    T = float(T) if T > 0 else float(L)
    if trunc:  # the rule looks at every intensity of [0, L]
        tab = rp_table(sigma_r, eps, L, T)
        N, C, idx = tab["N"], tab["C"], f.astype(np.int64)
    else:      # all 2N+1 terms: coefficients of the intensities present
        N = rp_order(T, sigma_r)
        vals, idx = np.unique(f, return_inverse=True)
        C = rp_coefs(N, sigma_r, L, vals)
        idx = idx.reshape(f.shape)
    J = C.shape[1] - 1
    x = to_unit(f, L)
    P = np.zeros_like(f)
    Q = np.zeros_like(f)
    for j in range(J + 1):
        G = npcheb.chebval(x, np.eye(J + 1)[j])          # phi_j(f)
        Fb = _o.blur_2d(f * G, op, sigma_s, R)           # S[F_j]
        Gb = _o.blur_2d(G, op, sigma_s, R)               # S[G_j]
        cj = C[idx, j]                                    # c_j(f(x))
        P += cj * Fb
        Q += cj * Gb
    ok = Q > 0
    out = np.where(ok, P / np.where(ok, Q, 1.0), f)
    return dict(out=out, N=N, J=J, n_nonpos=int((~ok).sum()), P=P, Q=Q)


def rp_direct_at(f, op, sigma_s: float, R: int, sigma_r: float, eps: float, L: float, ys, xs, T: float = 0.0):
    """Eq. (BF) evaluated directly at pixels (ys, xs) with the truncated
    polynomial kernel and the pointwise FIR or box spatial weights over the
    (2R+1)^2 window clipped to the image."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    T = float(T) if T > 0 else float(L)
    tab = rp_table(sigma_r, eps, L, T)
    d = np.arange(-R, R + 1)
    w1 = np.ones(2 * R + 1) if op == "box" else np.exp(-d * d / (2.0 * sigma_s * sigma_s))
    out = np.empty(len(ys))
    for i, (y, x) in enumerate(zip(ys, xs)):
        y0, y1, x0, x1 = max(0, y - R), min(H, y + R + 1), max(0, x - R), min(W, x + R + 1)
        win = f[y0:y1, x0:x1]
        w = np.outer(w1[y0 - y + R:y1 - y + R], w1[x0 - x + R:x1 - x + R])
        k = rp_kernel_trunc(win, np.full(win.shape, f[y, x]), tab["C"], tab["values"], L)
        num, den = float((w * k * win).sum()), float((w * k).sum())
        out[i] = num / den if den > 0 else f[y, x]
    return out
