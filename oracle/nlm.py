"""FP64 oracle of the shiftable non-local means of the paper's closing section.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper extends the method to the O(1) non-local means of its reference
[Kc2011]: with a small patch neighbourhood u_1 = 0, u_2, ..., u_p, the filter
is the ratio of the sums eq. (NL1) and eq. (NL2),

    NL1(x) = sum_{|y| <= R} f(x - y) g(s_1, ..., s_p),
    NL2(x) = sum_{|y| <= R}          g(s_1, ..., s_p),
    s_k    = f(x + u_k) - f(x - y + u_k),

with g an anisotropic Gaussian with diagonal covariance, each component
approximated by the raised cosine and truncated as for the bilateral filter
(Section 3), on [-T, T] with T from Algorithm 1.  The product of p expansions
has order N^p.

Readings (the paper is silent on them):

* The window is the square |y_1|, |y_2| <= R, and the sums run over the
  pixels x - y inside the image (the bilateral filter's zero extension); the
  sums carry no spatial weight ("box"), as eqs. (NL1), (NL2) are written, and
  the sampled Gaussian FIR weights are the other choice offered.
* Patch samples x + u_k outside the image take the nearest pixel (clamped
  coordinates).  Clamping moves both samples of s_k by at most |y| per
  coordinate, so |s_k| <= T still holds.
* Equal variances (sigma_r for every component): one order N and truncation
  M for all of them, from T and sigma_r by Algorithm 2 steps 3 and 4.
* A non-positive NL2 gives the input pixel (counted), as for the bilateral
  filter.

The result has a plain definition -- eqs. (NL1), (NL2) with the product of
truncated kernels phi_eps (eq. (approx)) -- which `nlm_direct` evaluates;
`nlm_shiftable` runs the expansion the GPU path runs (one term per
multi-index of kept frequencies, folded in conjugate pairs) and is pinned to
it.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import oracle as _o


def patch_stack(f, offsets):
    """(p, H, W): f at x + u_k, coordinates clamped into the image."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    ys, xs = np.mgrid[0:H, 0:W]
    return np.stack([f[np.clip(ys + dy, 0, H - 1), np.clip(xs + dx, 0, W - 1)] for dy, dx in offsets])


def kept_terms(N: int, M: int):
    """Kept n = M..N-M with weights 2^-N C(N, n) and m = 2n - N (eq. (approx))."""
    n = np.arange(M, N - M + 1)
    w = np.array([math.exp(math.lgamma(N + 1) - math.lgamma(k + 1) - math.lgamma(N - k + 1) - N * math.log(2.0))
                  for k in n])
    return 2 * n - N, w


def phi_table(N: int, M: int, sigma_r: float, smax: int):
    """phi_eps(s) for the integers s = -smax..smax (index s + smax)."""
    m, w = kept_terms(N, M)
    s = np.arange(-smax, smax + 1, dtype=np.float64)
    om = m / (math.sqrt(N) * sigma_r)
    return (w[None, :] * np.cos(s[:, None] * om[None, :])).sum(1)


def _weights(op, sigma_s: float, R: int):
    d = np.arange(-R, R + 1)
    return np.ones(2 * R + 1) if op == "box" else np.exp(-d * d / (2.0 * sigma_s * sigma_s))


def nlm_direct(f, offsets, op, sigma_s: float, R: int, N: int, M: int, sigma_r: float, smax: int = 255):
    """Eqs. (NL1)/(NL2) evaluated directly with the truncated product kernel
    (integer images).  Returns (out, NL1, NL2, n_nonpos)."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    P = patch_stack(f, offsets).astype(np.int64)
    tab = phi_table(N, M, sigma_r, smax)
    w1 = _weights(op, sigma_s, R)
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            # neighbour z = x - y with y = (dy, dx); only z inside the image
            y0, y1 = max(0, dy), min(H, H + dy)
            x0, x1 = max(0, dx), min(W, W + dx)
            if y0 >= y1 or x0 >= x1:
                continue
            k = np.full((y1 - y0, x1 - x0), w1[dy + R] * w1[dx + R])
            for c in range(P.shape[0]):
                s = P[c, y0:y1, x0:x1] - P[c, y0 - dy:y1 - dy, x0 - dx:x1 - dx]
                k = k * tab[s + smax]
            num[y0:y1, x0:x1] += k * f[y0 - dy:y1 - dy, x0 - dx:x1 - dx]
            den[y0:y1, x0:x1] += k
    ok = den > 0
    out = np.where(ok, num / np.where(ok, den, 1.0), f)
    return out, num, den, int((~ok).sum())


def multi_indices(N: int, M: int, p: int):
    """One multi-index m = (m_1..m_p) of kept frequencies from each conjugate
    pair {m, -m} (the one whose first non-zero component is negative), and the
    zero multi-index when N is even; weight 2 prod c (1 for the zero one)."""
    m1, w1 = kept_terms(N, M)
    wt = dict(zip(m1.tolist(), w1.tolist()))
    out = []
    for mv in itertools.product(m1.tolist(), repeat=p):
        nz = [v for v in mv if v != 0]
        if nz and nz[0] > 0:
            continue
        c = float(np.prod([wt[v] for v in mv]))
        out.append((mv, c if not nz else 2.0 * c))
    return out


def pair_count(N: int, M: int, p: int) -> int:
    """Multi-indices after folding: (L^p + z) / 2 with L = N - 2M + 1 kept
    terms per component and z = 1 when the zero multi-index exists (N even)."""
    L = N - 2 * M + 1
    return (L ** p + (1 if N % 2 == 0 else 0)) // 2


def nlm_shiftable(f, offsets, op, sigma_s: float, R: int, N: int, M: int, sigma_r: float):
    """The expansion: cos(sum_k w_k s_k) = cos(Th(x) - Th(x - y)) with the
    phase image Th_m(z) = alpha sum_k m_k f(z + u_k), alpha = 1/(sqrt(N)
    sigma_r); for each multi-index the images f cos Th, f sin Th, cos Th,
    sin Th are smoothed by the window operator and combined as in eqs. (f1),
    (f2).  Returns (out, NL1, NL2, n_nonpos)."""
    f = np.asarray(f, dtype=np.float64)
    P = patch_stack(f, offsets)
    alpha = 1.0 / (math.sqrt(N) * sigma_r)
    num = np.zeros_like(f)
    den = np.zeros_like(f)
    for mv, c in multi_indices(N, M, len(offsets)):
        th = alpha * np.tensordot(np.array(mv, dtype=np.float64), P, axes=1)
        cs, sn = np.cos(th), np.sin(th)
        num += c * (cs * _o.blur_2d(f * cs, op, sigma_s, R) + sn * _o.blur_2d(f * sn, op, sigma_s, R))
        den += c * (cs * _o.blur_2d(cs, op, sigma_s, R) + sn * _o.blur_2d(sn, op, sigma_s, R))
    ok = den > 0
    out = np.where(ok, num / np.where(ok, den, 1.0), f)
    return out, num, den, int((~ok).sum())


def nlm_algorithm(f, offsets, op, sigma_s: float, R: int, sigma_r: float, eps: float, range_: float = 255.0,
                  t_local: bool = True, t_value: float = 0.0, ys=None, xs=None):
    """T (Algorithm 1 with the window R, or the given global T), N and M
    (Algorithm 2 steps 3 and 4), then eqs. (NL1)/(NL2) directly.  With ys, xs
    only those pixels are returned (the whole image is still summed)."""
    f = np.asarray(f, dtype=np.float64)
    T = _o.range_T(f, R) if t_local else (t_value if t_value > 0 else range_)
    Tu = int(math.ceil(T))
    N = _o.order(Tu, sigma_r)
    M = _o.trunc_rule(N, sigma_r * 255.0 / range_, eps)
    out, num, den, bad = nlm_direct(f, offsets, op, sigma_s, R, N, M, sigma_r, smax=int(range_))
    res = dict(out=out, T=T, N=N, M=M, n_nonpos=bad, pairs=pair_count(N, M, len(offsets)))
    if ys is not None:
        res["out"] = out[ys, xs]
    return res
