"""CPU tests of libbf.so's host code (order tables, recursive-filter constants)
and a numpy model of the blocked recursive filter the kernels run, all checked
against the FP64 oracle.  The host code is compiled with g++ into a test shim;
no GPU is used."""
import ctypes
import math
import os
import subprocess
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM_DIR = os.path.join(ROOT, "tests", "_build")
SHIM = os.path.join(SHIM_DIR, "libtableshim.so")


@pytest.fixture(scope="module")
def shim():
    os.makedirs(SHIM_DIR, exist_ok=True)
    srcs = [os.path.join(ROOT, "tests", "table_shim.cpp"),
            os.path.join(ROOT, "paper_1203_5128_amd", "csrc", "bf_tables.cpp")]
    # built under a name of this process, then renamed, so that parallel
    # test workers never load a half-written library
    tmp = f"{SHIM}.{os.getpid()}"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "include")] + srcs + ["-o", tmp])
    os.replace(tmp, SHIM)
    L = ctypes.CDLL(SHIM)
    L.shim_order_N.argtypes = [ctypes.c_double, ctypes.c_double]
    L.shim_trunc_M.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
    P = ctypes.c_void_p
    L.shim_table_entry.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
    L.shim_iir_consts.argtypes = [ctypes.c_double, P, ctypes.c_int]
    L.shim_rp_table.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                P, P, P, P, P, P, ctypes.c_int]
    L.shim_layout.argtypes = [ctypes.c_int, P]
    return L


def entry(L, sigma_r, eps, rng_, T_cap, T):
    N, M, K = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    q = ctypes.c_ulonglong()
    at = ctypes.c_double()
    pm = (ctypes.c_int * 8192)()
    pc = (ctypes.c_float * 8192)()
    kmax = L.shim_table_entry(sigma_r, eps, rng_, T_cap, T, ctypes.byref(N), ctypes.byref(M), ctypes.byref(K),
                              ctypes.byref(q), ctypes.byref(at), pm, pc, 8192)
    assert kmax >= 0
    return dict(N=N.value, M=M.value, K=K.value, qfix=q.value, at=at.value,
                pm=np.array(pm[:K.value]), pc=np.array(pc[:K.value]), K_max=kmax)


def test_order_matches_oracle(shim):
    for sr in (2.0, 5.0, 10.0, 10.5, 20.0, 30.0, 60.0, 800.0, 1000.0):
        for T in list(range(0, 300)) + list(range(300, 65536, 997)):
            assert shim.shim_order_N(float(T), sr) == o.order(T, sr), (T, sr)


def test_truncation_matches_oracle(shim):
    for eps in (1e-2, 1e-3, 1e-4, 0.05):
        for sr8 in (5.0, 10.0, 10.01, 25.0, 40.0, 40.5):
            for N in list(range(1, 300)) + [411, 1053, 2718]:
                if 10.0 < sr8 <= 40.0 and N > 600:
                    continue
                assert shim.shim_trunc_M(N, sr8, eps) == o.trunc_rule(N, sr8, eps), (N, sr8, eps)


@pytest.mark.parametrize("sr,eps,rng_,T", [(10.0, 1e-3, 255.0, 212), (30.0, 1e-3, 255.0, 255),
                                           (20.0, 1e-3, 255.0, 255), (800.0, 1e-4, 65535.0, 65535),
                                           (50.0, 1e-3, 255.0, 100), (3.0, 1e-2, 255.0, 17)])
def test_pairs_match_expansion(shim, sr, eps, rng_, T):
    e = entry(shim, sr, eps, rng_, int(rng_), T)
    N = o.order(T, sr)
    M = o.trunc_rule(N, sr * 255.0 / rng_, eps)
    assert (e["N"], e["M"]) == (N, M)
    ns = [n for n in range(M, N - M + 1) if 2 * n < N]
    exp_m = [2 * n - N for n in ns] + ([0] if N % 2 == 0 else [])
    exp_c = [2 * o.coef(N, n) for n in ns] + ([o.coef(N, N // 2)] if N % 2 == 0 else [])
    assert list(e["pm"]) == exp_m
    assert np.allclose(e["pc"], exp_c, rtol=2e-7, atol=0)
    # the folded weights sum to the kept mass of eq. (approx)
    kept = sum(o.coef(N, n) for n in range(M, N - M + 1))
    assert abs(float(np.sum(e["pc"].astype(np.float64))) - kept) < 1e-5
    # fixed-point phase step: frac(1/(2 pi sqrt(N) sigma_r)) * 2^64 to a few units
    getcontext().prec = 60
    pi = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
    at = Decimal(1) / (2 * pi * Decimal(N).sqrt() * Decimal(repr(sr)))
    exact = (at - int(at)) * (Decimal(2) ** 64)
    assert abs(Decimal(e["qfix"]) - exact) < 64
    assert math.isclose(e["at"], float(at), rel_tol=1e-15)


# ------------------------------------------------------------------ IIR model
def consts(L, sigma, c=32):
    buf = (ctypes.c_float * 16384)()
    n = L.shim_iir_consts(sigma, buf, 16384)
    assert 0 < n <= 16384
    lay = (ctypes.c_int * 8)()
    L.shim_layout(c, lay)
    names = ["coef", "mts", "apow", "size", "kC", "lane", "scan", "wave"]
    lay = dict(zip(names, list(lay)))
    assert n == lay["size"]
    C = np.array(buf[:n], dtype=np.float64)
    kC = lay["kC"]
    # slot 0 holds 1 - g1: the first-order section runs without its input gain
    # g1 (kept in slot 3), so every pass scales its output by 1/g1
    return dict(a1=C[0], g2=C[1], c2=C[2], g1=C[3], kC=kC,
                mts=C[lay["mts"]:lay["mts"] + 9].reshape(3, 3),
                apow=C[lay["apow"]:lay["apow"] + 9 * (kC + 1)].reshape(kC + 1, 3, 3),
                lane=C[lay["lane"]:lay["lane"] + 9 * 64].reshape(64, 3, 3),
                scan=C[lay["scan"]:lay["scan"] + 9 * 8].reshape(8, 3, 3),
                wave=C[lay["wave"]:lay["wave"] + 9].reshape(3, 3))


def _sweep(x, st, a1, g2, c2, rev=False):
    s, w, d = st
    out = np.zeros_like(x)
    idx = range(len(x) - 1, -1, -1) if rev else range(len(x))
    for i in idx:
        s = a1 * s + x[i]
        d = (s - w) - c2 * d
        w = w + g2 * d
        out[i] = w
    return out, np.array([s, w, d])


def _scan_up(v, S, SW, off, A):
    """Inclusive scan of the chunk states across each row group as the kernel
    does it: Hillis-Steele inside 16-lane rows (row shifts), then the totals
    of rows 0 and 2 into rows 1 and 3 (row broadcast of lane 15) and, for 64
    lanes, of lanes 0..31 into rows 2 and 3 (broadcast of lane 31), each with
    the receiving lane's own power A^{c m} (A[m]).  A group of S < 64 threads
    starts at wave lane off."""
    v = [x.copy() for x in v]
    lane = [(off + t) % 64 if S <= 64 else t % 64 for t in range(S)]
    for d in (1, 2, 4, 8):
        if d >= SW:
            break
        o = [np.zeros(3)] * S
        for t in range(S):
            if lane[t] % 16 >= d and t % SW >= d:
                o[t] = v[t - d]
        v = [v[t] + A[d] @ o[t] for t in range(S)]
    if SW >= 32:
        o = [np.zeros(3)] * S
        for t in range(S):
            if (lane[t] >> 4) in (1, 3):
                o[t] = v[t - (lane[t] % 16) - 1]
        v = [v[t] + A[lane[t] % 16 + 1] @ o[t] for t in range(S)]
    if SW == 64:
        o = [np.zeros(3)] * S
        for t in range(S):
            if lane[t] >= 32:
                o[t] = v[t - lane[t] + 31]
        v = [v[t] + A[max(lane[t] - 31, 0)] @ o[t] for t in range(S)]
    return v


def _scan_down(v, S, SW, off, A):
    """The mirror image: row shifts the other way, then the totals of rows 1
    and 3 (from their first lane) into rows 0 and 2, and of lanes 32..63 into
    rows 0 and 1."""
    v = [x.copy() for x in v]
    lane = [(off + t) % 64 if S <= 64 else t % 64 for t in range(S)]
    for d in (1, 2, 4, 8):
        if d >= SW:
            break
        o = [np.zeros(3)] * S
        for t in range(S):
            if lane[t] % 16 + d <= 15 and t % SW + d < SW:
                o[t] = v[t + d]
        v = [v[t] + A[d] @ o[t] for t in range(S)]
    if SW >= 32:
        o = [np.zeros(3)] * S
        for t in range(S):
            if (lane[t] >> 4) in (0, 2):
                o[t] = v[t + 16 - lane[t] % 16]
        v = [v[t] + A[16 - lane[t] % 16] @ o[t] for t in range(S)]
    if SW == 64:
        o = [np.zeros(3)] * S
        for t in range(S):
            if lane[t] < 32:
                o[t] = v[t + 32 - lane[t]]
        v = [v[t] + A[max(32 - lane[t], 0)] @ o[t] for t in range(S)]
    return v


def model_blocked(x, C, off=0, tail=None):
    """Both recursive-pass kernels on one line (a row, or a column): per-thread
    sweeps from rest, scans of the chunk states across each wave's row group
    (_scan_up, _scan_down), wave carries through LDS, corrections with the w
    row of A^i.  tail=None: the line runs to the group's end (zero samples
    after it).  tail=array: the line ends with the last thread holding
    samples (as the horizontal pass for 8-bit and float rows) and the threads
    after it take these samples instead of zeros, which must reach no one."""
    kC = C["kC"]
    W = len(x)
    S = 1
    while S * kC < W:
        S *= 2
    SW = min(S, 64)
    if S > 32:
        off = 0
    off = off % 64 // SW * SW if SW < 64 else 0
    xp = np.zeros(S * kC)
    xp[:W] = x
    tlast = S - 1
    if tail is not None:
        tlast = (W + kC - 1) // kC - 1
        xp[(tlast + 1) * kC:] = tail[:(S - tlast - 1) * kC]
    a1, g2, c2 = C["a1"], C["g2"], C["c2"]
    A = C["lane"]
    zero3 = np.zeros(3)
    wt, tau = [], []
    for t in range(S):
        w, st = _sweep(xp[t * kC:(t + 1) * kC], zero3, a1, g2, c2)
        wt.append(w)
        tau.append(st)
    inc = _scan_up(tau, S, SW, off, A)
    exc = [np.zeros(3) if t % SW == 0 else inc[t - 1] for t in range(S)]
    if S > 64:
        NW = S // 64
        tot = [inc[w * 64 + 63] for w in range(NW)]
        for t in range(S):
            wig, ls = t // 64, t % 64
            Kc = np.zeros(3)
            for w in range(wig):
                Kc = tot[w] + C["wave"] @ Kc
            exc[t] = exc[t] + A[ls] @ Kc
            if t == tlast:  # the carry through its own chunk too
                inc[t] = inc[t] + (A[ls + 1] if ls < 63 else C["wave"]) @ Kc
    for t in range(S):
        for i in range(kC):
            wt[t][i] += C["apow"][i + 1][1] @ exc[t]
    Eb = C["mts"] @ inc[tlast]
    zt, hd = [], []
    for t in range(S):
        z, st = _sweep(wt[t], zero3, a1, g2, c2, rev=True)
        zt.append(z)
        hd.append(st)
    hd = [h if t <= tlast else np.zeros(3) for t, h in enumerate(hd)]
    hd[tlast] = hd[tlast] + A[1] @ Eb
    hd = _scan_down(hd, S, SW, off, A)
    ein = [np.zeros(3) if t % SW == SW - 1 else hd[t + 1] for t in range(S)]
    if S > 64:
        NW = S // 64
        tot = [hd[w * 64] for w in range(NW)]
        for t in range(S):
            wig, ls = t // 64, t % 64
            Kc = np.zeros(3)
            for w in range(NW - 1, wig, -1):
                Kc = tot[w] + C["wave"] @ Kc
            ein[t] = ein[t] + A[63 - ls] @ Kc
    ein[tlast] = Eb
    for t in range(S):
        for i in range(kC):
            zt[t][i] += C["apow"][kC - i][1] @ ein[t]
    return np.concatenate(zt)[:W]


@pytest.mark.parametrize("c", [16, 32])
@pytest.mark.parametrize("sigma", [0.7, 3.0, 10.0, 16.0])
@pytest.mark.parametrize("n", [1, 7, 32, 33, 200, 300, 512, 1000, 2049, 4096, 8192])
def test_blocked_model_matches_oracle(shim, c, sigma, n):
    """The blocked filter of both passes (rows and columns, n up to the 8192
    limit) against the oracle's recursive Gaussian on the same line."""
    if c == 16 and n > 16 * 256:
        pytest.skip("lines longer than 4096 use the 32-sample chunk")
    C = consts(shim, sigma, c)
    rng = np.random.default_rng(1000 + n)
    x = rng.uniform(-1, 1, n)
    ref = o.blur_1d(x, "iir", sigma)
    for off in (0, 32, 48):  # where the row group sits in its wave
        got = model_blocked(x, C, off) * C["g1"] ** 2
        assert np.abs(got - ref).max() < 2e-5 * max(1.0, np.abs(ref).max()), off


@pytest.mark.parametrize("c", [16, 32])
@pytest.mark.parametrize("sigma", [3.0, 16.0])
@pytest.mark.parametrize("n", [7, 100, 300, 1030, 1040, 1500, 2064, 2100, 4100])
def test_blocked_model_line_end(shim, c, sigma, n):
    """A line that ends before its row group, the threads after it holding
    arbitrary samples: the oracle's recursive Gaussian, and the same outputs
    whatever those samples are.  n = 1040 and 2064 (16-sample chunks) end
    exactly at the first lane of a later wave, where the last thread's
    inclusive state takes the previous waves' carry through its own chunk."""
    if c == 16 and n > 16 * 256:
        pytest.skip("lines longer than 4096 use the 32-sample chunk")
    C = consts(shim, sigma, c)
    rng = np.random.default_rng(2000 + n)
    x = rng.uniform(-1, 1, n)
    tail = rng.uniform(-50, 50, 256 * c)
    ref = o.blur_1d(x, "iir", sigma)
    for off in (0, 32):
        got = model_blocked(x, C, off, tail=tail)
        zero = model_blocked(x, C, off, tail=np.zeros_like(tail))
        assert np.array_equal(got, zero), off
        assert np.abs(got * C["g1"] ** 2 - ref).max() < 2e-5 * max(1.0, np.abs(ref).max()), off


# ------------------------------------------------- polynomial range kernel
@pytest.mark.parametrize("sr,eps,T", [(30.0, 1e-3, 255.0), (10.0, 1e-3, 255.0), (20.0, 1e-2, 255.0),
                                      (60.0, 1e-4, 255.0), (25.0, 1e-3, 220.0), (5.0, 1e-3, 255.0)])
def test_polynomial_table_matches_oracle(shim, sr, eps, T):
    """The library's Chebyshev table (its own DCT in long double) against the
    oracle's (numpy interpolation in FP64): same order N and kept order J,
    basis values T_j(x(v)) and coefficients c_j(v) to FP32 rounding."""
    from oracle import poly as rp
    cap = 2 * 256 * 2048
    N, J, K = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    kap = ctypes.c_double()
    gen = (ctypes.c_float * cap)()
    comb = (ctypes.c_float * cap)()
    n = shim.shim_rp_table(sr, eps, 255.0, T, ctypes.byref(N), ctypes.byref(J), ctypes.byref(K), ctypes.byref(kap),
                           gen, comb, cap)
    assert n == K.value * 512
    tab = rp.rp_table(sr, eps, 255.0, T)
    assert (N.value, J.value) == (tab["N"], tab["J"])
    assert K.value == (J.value + 2) // 2
    g = np.array(gen[:n]).reshape(K.value, 256, 2)
    c = np.array(comb[:n]).reshape(K.value, 256, 2)
    x = rp.to_unit(np.arange(256.0), 255.0)
    for j in range(J.value + 1):
        Tj = np.cos(j * np.arccos(x))
        assert np.abs(g[j // 2, :, j % 2] - Tj).max() <= 2e-7
        ref = tab["C"][:, j]
        assert np.abs(c[j // 2, :, j % 2] - ref).max() <= 1e-7 * max(1.0, np.abs(ref).max()) + 1e-9
    if J.value % 2 == 0:  # the unused half of the last slot carries no coefficient
        assert np.all(c[-1, :, 1] == 0.0)
    assert abs(kap.value - np.abs(tab["C"]).sum(1).max()) < 1e-6
