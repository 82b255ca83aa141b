"""GPU parity of the constant (box) spatial filter (Section 4: SHIFTABLE-BF
with a constant spatial filter and a Gaussian range kernel) against the FP64
oracle running the same operator.

The box runs on the Toeplitz kernels with unit taps over |j| <= R.  T, N, M
and the count of non-positive denominators must match exactly; the output
must lie within the variant's tolerance (2e-3 for the split FP16 variant).
"""
import numpy as np
import pytest

import oracle as o
from bfsynth import CONFIGS, config_image, gen_random

pytestmark = pytest.mark.gpu

U = {"toeplitz_f16": 2.0 ** -11, "toeplitz_bf16": 2.0 ** -8, "toeplitz_bf16x2": 2.0 ** -16,
     "toeplitz_f16x2": 0.0}
TOL = {b: max(2e-3, 2.0 ** 11 * u) for b, u in U.items()}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_box(img, dtype, blur, R, sigma_r, eps, t_mode="local", t_value=0.0):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    plan = Plan.create(make_params(H, W, dtype, sigma_s=float(R), sigma_r=sigma_r, eps=eps, radius=R,
                                   t_mode=t_mode, t_value=t_value, blur=blur, spatial="box"))
    out, rep = plan.filter(torch.from_numpy(np.ascontiguousarray(img)).to("cuda"))
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().astype(np.float64), rep


def compare(img, dtype, blur, R, sigma_r, eps, label=""):
    out, rep = run_box(img, dtype, blur, R, sigma_r, eps)
    rng_ = 65535.0 if dtype == "u16" else 255.0
    ref = o.algorithm2(img.astype(np.float64), "box", 1.0, R, sigma_r, eps, rng_, True)
    assert rep["T"] == ref["T"] and (rep["N"], rep["M"]) == (ref["N"], ref["M"])
    err = np.abs(out - ref["out"])
    tol = TOL[blur] * rng_ / 255.0
    print(f"[box] {label} {blur} {img.shape} {dtype} R={R} T={rep['T']} N={rep['N']} M={rep['M']} "
          f"pairs={rep['pairs']} max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e} tol={tol:.3e}", flush=True)
    assert rep["variant"] == blur
    assert err.max() <= tol
    assert rep["q_nonpos"] == ref["n_nonpos"]
    return out, rep, ref


@pytest.mark.parametrize("shape", [(1, 1), (1, 50), (50, 1), (33, 65), (100, 257), (130, 64)])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("blur", ["toeplitz_f16x2", "toeplitz_bf16x2", "toeplitz_f16"])
def test_small_parity(blur, dtype, shape):
    img = gen_random(900 + 7 * shape[0] + shape[1], *shape, dtype=dtype)
    sc = 257.0 if dtype == "u16" else 1.0
    compare(img, dtype, blur, 3, 25.0 * sc, 1e-2, label="small")


@pytest.mark.parametrize("R", [1, 2, 5, 10, 14, 20, 48, 120])
def test_radii(R):
    """The radii of the paper's run-time comparison (2..20) and beyond, at
    eps = 0.01."""
    img = gen_random(950 + R, 80, 300, dtype="u8")
    compare(img, "u8", "toeplitz_f16x2", R, 10.0, 1e-2, label=f"R={R}")


@pytest.mark.parametrize("sigma_r", [5.0, 10.0, 30.0])
def test_paper_setting_grad512_sampled(sigma_r):
    """512 x 512 (the gradient workload image), box radius 20, eps = 0.01 (the
    setting of the paper's comparison with integral histograms at sigma_r = 5):
    T, N, M exactly, the output at sampled pixels against eq. (BF) evaluated
    directly with the box filter."""
    c = CONFIGS[2]
    img = config_image(2)
    R = 20
    out, rep = run_box(img, "u8", "toeplitz_f16x2", R, sigma_r, 1e-2)
    f = img.astype(np.float64)
    T = o.range_T(f, R)
    N = o.order(T, sigma_r)
    M = o.trunc_rule(N, sigma_r, 1e-2)
    assert rep["T"] == T and (rep["N"], rep["M"]) == (N, M)
    rng = np.random.default_rng(71)
    ys = np.concatenate([rng.integers(0, 512, 200), [0, 0, 511, 511, 256]])
    xs = np.concatenate([rng.integers(0, 512, 200), [0, 511, 0, 511, 3]])
    ref = o.direct_box_at(f, R, N, M, sigma_r, ys, xs)
    err = np.abs(out[ys, xs] - ref)
    print(f"[box] grad512 R=20 sr={sigma_r} T={T} N={N} M={M} pairs={rep['pairs']} sampled max={err.max():.3e}",
          flush=True)
    assert err.max() <= 2e-3


def test_constant_image_unchanged():
    for v, dt in ((0, "u8"), (200, "u8"), (40000, "u16"), (77.25, "f32")):
        img = np.full((40, 70), v, dtype={"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[dt])
        sc = 257.0 if dt == "u16" else 1.0
        out, rep = run_box(img, dt, "toeplitz_f16x2", 4, 20.0 * sc, 1e-2)
        assert rep["T"] == 0 and rep["N"] == 1
        assert np.abs(out - float(v)).max() <= 2e-3 * sc


def test_batch_mixes_box_and_gaussian_images():
    """Box and Gaussian images in one grouped batch: each output equals the
    image filtered alone by its own plan, and the oracle with its operator."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    items = [(gen_random(990 + i, 60 + 17 * i, 90 + 11 * i, dtype="u8"), kind, R)
             for i, (kind, R) in enumerate([("box", 2), ("gaussian", 6), ("box", 9), ("box", 20), ("gaussian", 9)])]
    params = [make_params(im.shape[0], im.shape[1], "u8", sigma_s=(R if k == "box" else R / 3.0), sigma_r=15.0,
                          eps=1e-2, radius=R, blur="toeplitz_f16x2", spatial=k) for im, k, R in items]
    plan = Plan.create(params)
    outs, reps = plan.filter_batch([torch.from_numpy(im).to("cuda") for im, _, _ in items])
    torch.cuda.synchronize()
    plan.close()
    for (im, kind, R), p, out, rep in zip(items, params, outs, reps):
        single = Plan.create(p)
        alone, _ = single.filter(torch.from_numpy(im).to("cuda"))
        torch.cuda.synchronize()
        single.close()
        got = out.cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy()), (kind, R)
        op = "box" if kind == "box" else "fir"
        ref = o.algorithm2(im.astype(np.float64), op, (1.0 if kind == "box" else R / 3.0), R, 15.0, 1e-2, 255.0,
                           True)
        err = np.abs(got.astype(np.float64) - ref["out"]).max()
        print(f"[box] batch {kind} R={R} {im.shape} max={err:.3e}", flush=True)
        assert err <= 2e-3
