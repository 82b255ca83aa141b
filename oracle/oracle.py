"""Python side of the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two kinds of code live here:

* ctypes bindings to ``bf_oracle.c`` (the step-by-step FP64 implementation of
  Algorithm 2 of the paper, with both spatial operators);
* small, independent definitions used to pin that C code: brute-force window
  extrema, exact rational arithmetic for the order/truncation rules, and the
  direct (non-expanded) bilateral filter of eq. (BF) with a materialised
  spatial operator.

Paper citations name the section, equation, algorithm or table.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bf_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

OP_FIR = 0
OP_IIR = 1
OP_BOX = 2
_OPS = {"fir": OP_FIR, "iir": OP_IIR, "box": OP_BOX, OP_FIR: OP_FIR, OP_IIR: OP_IIR, OP_BOX: OP_BOX}

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, OpenMP, IEEE semantics)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        D = ctypes.c_double
        I = ctypes.c_int
        Lg = ctypes.c_long
        P = ctypes.c_void_p
        L.orc_maxfilter_1d.argtypes = [P, Lg, Lg, P]
        L.orc_range_T.argtypes = [P, Lg, Lg, Lg, P, P]
        L.orc_order.argtypes = [D, D]
        L.orc_order.restype = I
        L.orc_coef.argtypes = [I, I]
        L.orc_coef.restype = D
        L.orc_trunc_exact.argtypes = [I, D]
        L.orc_trunc_exact.restype = I
        L.orc_trunc_chernoff.argtypes = [I, D]
        L.orc_trunc_chernoff.restype = I
        L.orc_trunc_rule.argtypes = [I, D, D]
        L.orc_trunc_rule.restype = I
        L.orc_phi.argtypes = [D, I, D]
        L.orc_phi.restype = D
        L.orc_phi_eps.argtypes = [D, I, I, D]
        L.orc_phi_eps.restype = D
        L.orc_yvv_coefs.argtypes = [D, P]
        L.orc_blur_1d.argtypes = [P, Lg, I, D, Lg, P]
        L.orc_blur_2d.argtypes = [P, Lg, Lg, I, D, Lg]
        L.orc_shiftable_bf.argtypes = [P, Lg, Lg, I, D, Lg, I, I, D, P, P, P, P]
        L.orc_algorithm2.argtypes = [P, Lg, Lg, I, D, Lg, D, D, D, I, D, P, P, P, P, P]
        L.orc_direct_fir_at.argtypes = [P, Lg, Lg, D, Lg, I, I, D, P, P, Lg, P]
        L.orc_direct_at.argtypes = [P, Lg, Lg, I, D, Lg, I, I, D, P, P, Lg, P]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")


# ---------------------------------------------------------------- Algorithm 1
def maxfilter_1d(x, R: int) -> np.ndarray:
    """Appendix MAX-FILTER: windowed maximum over [i-R, i+R], clipped."""
    x = _f64(x)
    out = np.empty_like(x)
    _check(lib().orc_maxfilter_1d(_ptr(x), x.size, int(R), _ptr(out)))
    return out


def range_T(f, R: int, return_map: bool = False):
    """Algorithm 1: T = max_x [max_{window} f - f(x)]."""
    f = _f64(f)
    H, W = f.shape
    Mx = np.empty_like(f)
    T = ctypes.c_double()
    _check(lib().orc_range_T(_ptr(f), H, W, int(R), _ptr(Mx), ctypes.byref(T)))
    return (T.value, Mx) if return_map else T.value


def brute_window_extrema(f, R: int):
    """Brute-force max and min of f over the clipped (2R+1)^2 square window."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    mx = np.full((H, W), -np.inf)
    mn = np.full((H, W), np.inf)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            ys0, ys1 = max(0, -dy), min(H, H - dy)
            xs0, xs1 = max(0, -dx), min(W, W - dx)
            if ys0 >= ys1 or xs0 >= xs1:
                continue
            src = f[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
            mx[ys0:ys1, xs0:xs1] = np.maximum(mx[ys0:ys1, xs0:xs1], src)
            mn[ys0:ys1, xs0:xs1] = np.minimum(mn[ys0:ys1, xs0:xs1], src)
    return mx, mn


def brute_T(f, R: int) -> float:
    """Eq. (bound) by brute force: max_x max_{|y|<=R} |f(x-y) - f(x)|."""
    f = np.asarray(f, dtype=np.float64)
    mx, mn = brute_window_extrema(f, R)
    return float(max((mx - f).max(), (f - mn).max()))


# ------------------------------------------------- order and truncation rules
def order(T: float, sigma_r: float) -> int:
    return int(lib().orc_order(float(T), float(sigma_r)))


def coef(N: int, n: int) -> float:
    return float(lib().orc_coef(int(N), int(n)))


def trunc_exact(N: int, eps: float) -> int:
    return int(lib().orc_trunc_exact(int(N), float(eps)))


def trunc_chernoff(N: int, eps: float) -> int:
    return int(lib().orc_trunc_chernoff(int(N), float(eps)))


def trunc_rule(N: int, sigma_r8: float, eps: float) -> int:
    return int(lib().orc_trunc_rule(int(N), float(sigma_r8), float(eps)))


def phi(s: float, N: int, sigma_r: float) -> float:
    return float(lib().orc_phi(float(s), int(N), float(sigma_r)))


def phi_eps(s: float, N: int, M: int, sigma_r: float) -> float:
    return float(lib().orc_phi_eps(float(s), int(N), int(M), float(sigma_r)))


def yvv_coefs(sigma: float):
    c = np.zeros(4)
    lib().orc_yvv_coefs(float(sigma), _ptr(c))
    return c


# Exact rational versions, used only as pins for the C code above.
def exact_cum(N: int, m: int) -> Fraction:
    """sum_{n=0}^{m} C(N,n) / 2^N, exactly."""
    s = 0
    c = 1
    for n in range(0, m + 1):
        s += c
        c = c * (N - n) // (n + 1)
    return Fraction(s, 2 ** N)


def exact_trunc(N: int, eps: float) -> int:
    """Smallest m with sum_{n<=m} C(N,n)/2^N > eps/2, in exact arithmetic."""
    half = Fraction(eps) / 2
    s = 0
    c = 1
    tot = 2 ** N
    for m in range(N + 1):
        s += c
        if Fraction(s, tot) > half:
            return m
        c = c * (N - m) // (m + 1)
    return N // 2


# ---------------------------------------------------------- spatial operators
def blur_1d(x, op, sigma: float, R: int = 0) -> np.ndarray:
    x = _f64(x)
    out = np.empty_like(x)
    _check(lib().orc_blur_1d(_ptr(x), x.size, _OPS[op], float(sigma), int(R), _ptr(out)))
    return out


def blur_2d(img, op, sigma: float, R: int = 0) -> np.ndarray:
    a = _f64(img).copy()
    H, W = a.shape
    _check(lib().orc_blur_2d(_ptr(a), H, W, _OPS[op], float(sigma), int(R)))
    return a


def operator_matrix(n: int, op, sigma: float, R: int = 0) -> np.ndarray:
    """The 1-D operator as an n x n matrix: column j is the response to e_j."""
    S = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        S[:, j] = blur_1d(e, op, sigma, R)
    return S


# ------------------------------------------------------------- the filter
def shiftable_bf(f, op, sigma_s: float, R: int, N: int, M: int, sigma_r: float):
    """SHIFTABLE-BF with the truncated kernel; returns (out, P, Q, n_nonpos)."""
    f = _f64(f)
    H, W = f.shape
    out = np.empty_like(f)
    P = np.empty_like(f)
    Q = np.empty_like(f)
    bad = ctypes.c_long()
    _check(lib().orc_shiftable_bf(_ptr(f), H, W, _OPS[op], float(sigma_s), int(R), int(N), int(M),
                                  float(sigma_r), _ptr(out), _ptr(P), _ptr(Q), ctypes.byref(bad)))
    return out, P, Q, bad.value


def algorithm2(f, op, sigma_s: float, R: int, sigma_r: float, eps: float, range_: float,
               t_local: bool, t_value: float = 0.0):
    """Algorithm 2 end to end; returns dict(out, T, N, M, n_nonpos)."""
    f = _f64(f)
    H, W = f.shape
    out = np.empty_like(f)
    T = ctypes.c_double()
    N = ctypes.c_int()
    M = ctypes.c_int()
    bad = ctypes.c_long()
    _check(lib().orc_algorithm2(_ptr(f), H, W, _OPS[op], float(sigma_s), int(R), float(sigma_r),
                                float(eps), float(range_), int(bool(t_local)), float(t_value),
                                _ptr(out), ctypes.byref(T), ctypes.byref(N), ctypes.byref(M),
                                ctypes.byref(bad)))
    return dict(out=out, T=T.value, N=N.value, M=M.value, n_nonpos=bad.value)


def direct_fir_at(f, sigma_s: float, R: int, N: int, M: int, sigma_r: float, ys, xs):
    """Eq. (BF) evaluated directly at the given pixels (FIR operator, phi_eps)."""
    f = _f64(f)
    H, W = f.shape
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int64))
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int64))
    out = np.empty(ys.size)
    _check(lib().orc_direct_fir_at(_ptr(f), H, W, float(sigma_s), int(R), int(N), int(M),
                                   float(sigma_r), _ptr(ys), _ptr(xs), ys.size, _ptr(out)))
    return out


def direct_box_at(f, R: int, N: int, M: int, sigma_r: float, ys, xs):
    """Eq. (BF) evaluated directly at the given pixels with the constant
    spatial filter of radius R (Section 4) and phi_eps."""
    f = _f64(f)
    H, W = f.shape
    ys = np.ascontiguousarray(np.asarray(ys, dtype=np.int64))
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int64))
    out = np.empty(ys.size)
    _check(lib().orc_direct_at(_ptr(f), H, W, OP_BOX, 1.0, int(R), int(N), int(M), float(sigma_r),
                               _ptr(ys), _ptr(xs), ys.size, _ptr(out)))
    return out


def direct_bf_dense(f, Sv: np.ndarray, Sh: np.ndarray, range_kernel) -> np.ndarray:
    """Eq. (BF) by brute force with a materialised separable operator.

    The weight of pixel y in the output at x is Sv[x1, y1] * Sh[x2, y2] times
    range_kernel(f(y) - f(x)).  Tiny images only (O((HW)^2))."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    Wsp = np.einsum("ac,bd->abcd", Sv, Sh).reshape(H * W, H * W)
    fv = f.reshape(-1)
    K = Wsp * range_kernel(fv[None, :] - fv[:, None])
    num = K @ fv
    den = K.sum(axis=1)
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), fv)
    return out.reshape(H, W)


def phi_eps_vec(N: int, M: int, sigma_r: float):
    """Vectorised eq. (approx) written out independently of the C code."""
    n = np.arange(M, N - M + 1)
    logc = np.array([math.lgamma(N + 1) - math.lgamma(k + 1) - math.lgamma(N - k + 1)
                     for k in n]) - N * math.log(2.0)
    c = np.exp(logc)
    om = (2 * n - N) / (math.sqrt(N) * sigma_r)

    def k(s):
        s = np.asarray(s, dtype=np.float64)
        return (c[None, :] * np.cos(s.reshape(-1, 1) * om[None, :])).sum(1).reshape(s.shape)
    return k
