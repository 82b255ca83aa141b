"""GPU parity of the Toeplitz MFMA blur variants against the FP64 oracle with
the FIR operator (taps exp(-j^2 / 2 sigma_s^2), |j| <= R, zero extension).

T, N, M and the count of non-positive denominators must match exactly.  The
filtered image must lie within the variant's tolerance on the [0, 255] scale
(scaled by range/255 for 16-bit images).  Max and RMS errors are printed for
every case.
"""
import os

import numpy as np
import pytest

import oracle as o
from bfsynth import CONFIGS, config_image, gen_random

pytestmark = pytest.mark.gpu

VARIANTS = ["toeplitz_f16", "toeplitz_bf16", "toeplitz_f16x2", "toeplitz_bf16x2"]
# Max error on the [0, 255] scale: max(2e-3, 2^11 u) with u the unit
# roundoff of the variant's operands (2^-11 FP16, 2^-8 BF16, 2^-16 for a BF16
# hi + lo pair; an FP16 hi + lo pair carries 22 bits and is held to the FP32
# target).  Each output is a ratio of sums of products of rounded operands;
# its relative error is a few u times the conditioning of the denominator,
# which stays below 2^11 on every image here (adversarial noise at R = 120
# included) and far below it on the workloads.
U = {"toeplitz_f16": 2.0 ** -11, "toeplitz_bf16": 2.0 ** -8, "toeplitz_bf16x2": 2.0 ** -16,
     "toeplitz_f16x2": 0.0}
TOL = {b: max(2e-3, 2.0 ** 11 * u) for b, u in U.items()}
# The variants that meet the 2e-3 target on the workloads themselves.
TARGET = 2e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(img, dtype, blur, **kw):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    plan = Plan.create(make_params(H, W, dtype, blur=blur, **kw))
    t = torch.from_numpy(np.ascontiguousarray(img)).to("cuda")
    out, rep = plan.filter(t)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().astype(np.float64), rep


def compare(img, dtype, blur, sigma_s, sigma_r, eps, radius=0, t_mode="local", t_value=0.0, label=""):
    out, rep = run_gpu(img, dtype, blur, sigma_s=sigma_s, sigma_r=sigma_r, eps=eps, radius=radius,
                       t_mode=t_mode, t_value=t_value)
    rng_ = 65535.0 if dtype == "u16" else 255.0
    R = radius if radius > 0 else int(np.ceil(3 * sigma_s))
    ref = o.algorithm2(img.astype(np.float64), "fir", sigma_s, R, sigma_r, eps, rng_, t_mode == "local",
                       t_value if t_value > 0 else rng_)
    assert rep["T"] == ref["T"], (rep, ref["T"])
    assert (rep["N"], rep["M"]) == (ref["N"], ref["M"])
    err = np.abs(out - ref["out"])
    tol = TOL[blur] * (rng_ / 255.0)
    print(f"[toeplitz] {label} {blur} {img.shape} {dtype} R={R} T={rep['T']} N={rep['N']} M={rep['M']} "
          f"pairs={rep['pairs']} max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e} tol={tol:.3e} "
          f"qnp={rep['q_nonpos']}/{ref['n_nonpos']}", flush=True)
    assert rep["variant"] == blur
    assert err.max() <= tol
    assert rep["q_nonpos"] == ref["n_nonpos"]
    return out, rep, ref


SHAPES = [(1, 1), (17, 1), (1, 130), (33, 65), (100, 257), (130, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("blur", VARIANTS)
def test_small_parity(blur, dtype, shape):
    img = gen_random(11 * shape[0] + shape[1], *shape, dtype=dtype)
    sc = 257.0 if dtype == "u16" else 1.0
    compare(img, dtype, blur, 2.0, 25.0 * sc, 1e-3, label="small")


@pytest.mark.parametrize("R", [0, 1, 7, 8, 9, 15, 24, 31, 48, 57, 72, 104, 120])
@pytest.mark.parametrize("blur", VARIANTS)
def test_radii(blur, R):
    img = gen_random(500 + R, 90, 300, dtype="u8")
    compare(img, "u8", blur, max(R / 3.0, 0.6), 20.0, 1e-3, radius=R if R > 0 else 0, label=f"R={R}")


@pytest.mark.parametrize("width", [127, 128, 129, 4100, 9000])
@pytest.mark.parametrize("blur", ["toeplitz_f16", "toeplitz_f16x2"])
def test_widths(blur, width):
    img = gen_random(width, 20, width, dtype="u8")
    compare(img, "u8", blur, 3.0, 30.0, 1e-3, label=f"W={width}")


@pytest.mark.parametrize("blur", VARIANTS)
def test_global_mode(blur):
    img = gen_random(5, 80, 90, dtype="u8")
    compare(img, "u8", blur, 3.0, 30.0, 1e-3, t_mode="global", t_value=255.0, label="global")


@pytest.mark.parametrize("blur", ["toeplitz_f16", "toeplitz_bf16x2"])
def test_several_launches(blur):
    """A workspace budget below one pair's images forces one pair per launch, so
    the numerator and denominator accumulate across launches."""
    img = gen_random(77, 70, 150, dtype="u8")
    os.environ["BF_Z_BUDGET_MB"] = "0"
    try:
        compare(img, "u8", blur, 2.5, 12.0, 1e-3, label="multi-launch")
    finally:
        del os.environ["BF_Z_BUDGET_MB"]


def test_workload2_grad512_split():
    c = CONFIGS[2]
    img = config_image(2)
    out, rep, ref = compare(img, "u8", "toeplitz_f16x2", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"],
                            label="cfg2")
    assert np.abs(out - ref["out"]).max() <= TARGET


def sampled_compare(idx, dtype, blur, n=300):
    """Full-size workload: T exactly against Algorithm 1 on the host, the
    output at sampled pixels (corners and edges included) against eq. (BF)
    evaluated directly with the truncated kernel and the FIR operator."""
    c = CONFIGS[idx]
    img = config_image(idx)
    out, rep = run_gpu(img, dtype, blur, sigma_s=c["sigma_s"], sigma_r=c["sigma_r"], eps=c["eps"],
                       radius=c["radius"], t_mode="local")
    rng_ = 65535.0 if dtype == "u16" else 255.0
    f = img.astype(np.float64)
    T = o.range_T(f, c["radius"])
    N = o.order(T, c["sigma_r"])
    M = o.trunc_rule(N, c["sigma_r"] * 255.0 / rng_, c["eps"])
    assert rep["T"] == T and (rep["N"], rep["M"]) == (N, M)
    H, W = img.shape
    rng = np.random.default_rng(44 + idx)
    ys = np.concatenate([rng.integers(0, H, n), [0, 0, H - 1, H - 1, 5, H // 2]])
    xs = np.concatenate([rng.integers(0, W, n), [0, W - 1, 0, W - 1, W // 2, 3]])
    ref = o.direct_fir_at(f, c["sigma_s"], c["radius"], N, M, c["sigma_r"], ys, xs)
    err = np.abs(out[ys, xs] - ref)
    tol = TOL[blur] * rng_ / 255.0
    print(f"[toeplitz] cfg{idx} {blur} T={T} N={N} M={M} pairs={rep['pairs']} sampled max={err.max():.3e} "
          f"rms={np.sqrt((err ** 2).mean()):.3e} tol={tol:.3e}", flush=True)
    assert err.max() <= tol
    return err.max()


@pytest.mark.parametrize("blur", ["toeplitz_f16x2", "toeplitz_bf16x2"])
def test_workload3_poly2048_u16_sampled(blur):
    sampled_compare(3, "u16", blur)


@pytest.mark.parametrize("blur", VARIANTS)
def test_workload4_mosaic4096_sampled(blur):
    err = sampled_compare(4, "f32", blur)
    if blur.endswith("x2"):
        assert err <= TARGET


@pytest.mark.parametrize("blur", VARIANTS)
def test_constant_image_unchanged(blur):
    for v, dt in ((0, "u8"), (200, "u8"), (40000, "u16"), (77.25, "f32")):
        img = np.full((40, 70), v, dtype={"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[dt])
        sc = 257.0 if dt == "u16" else 1.0
        out, rep = run_gpu(img, dt, blur, sigma_s=3.0, sigma_r=20.0 * sc, eps=1e-3)
        assert rep["T"] == 0 and rep["N"] == 1
        assert np.abs(out - float(v)).max() <= TOL[blur] * sc


@pytest.mark.parametrize("blur", ["toeplitz_f16", "toeplitz_f16x2"])
def test_graph_replays_match_eager(blur):
    """Replays of the captured launch sequence, with eager work and
    synchronisations between them, equal the eager result bit for bit."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    img = gen_random(91, 120, 200, dtype="u8")
    x = torch.from_numpy(img).to("cuda")
    os.environ["BF_GRAPH"] = "0"
    try:
        pe = Plan.create(make_params(120, 200, "u8", sigma_s=3.0, sigma_r=15.0, blur=blur))
    finally:
        del os.environ["BF_GRAPH"]
    eager, _ = pe.filter(x)
    torch.cuda.synchronize()
    pe.close()
    pg = Plan.create(make_params(120, 200, "u8", sigma_s=3.0, sigma_r=15.0, blur=blur))
    out = torch.empty((120, 200), dtype=torch.float32, device="cuda")
    for _ in range(4):
        out.fill_(-1.0)
        pg.filter(x, out, report=False)
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        _ = (x.float() * 2).sum().item()
    pg.close()
