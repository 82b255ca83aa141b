"""GPU parity of the polynomial range kernel (eq. (RPconv), Section 1.3) in
its Chebyshev form, against the FP64 oracle running the same kernel,
truncation and spatial operator (oracle/poly.py): small shapes and ragged
tails on the recursive blur, the split Toeplitz blurs and the box filter, the
256x256 rectangles workload whole, a 512x512 image at sigma_r = 10 (N = 326)
at sampled pixels against eq. (BF) evaluated directly, and a batch that mixes
both range kernels (each output equal, bit for bit, to its single-image
plan)."""
import numpy as np
import pytest

from bfsynth import config_image, gen_random
from oracle import poly as rp

pytestmark = pytest.mark.gpu

OP = {"iir_f32": "iir", "toeplitz_f16x2": "fir", "toeplitz_bf16x2": "fir"}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params(H, W, ss, R, sr, eps, blur, spatial="gaussian", T=0.0):
    from paper_1203_5128_amd import make_params
    return make_params(H, W, "u8", sigma_s=ss, sigma_r=sr, eps=eps, radius=R, t_mode="global", t_value=T,
                       blur=blur, spatial=spatial, range_kernel="polynomial")


def _run(img, p):
    torch = _torch()
    from paper_1203_5128_amd import Plan
    plan = Plan.create(p)
    out, rep = plan.filter(torch.from_numpy(np.ascontiguousarray(img)).to("cuda"))
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().astype(np.float64), rep


def _check(img, out, rep, ref, tol=2e-3):
    assert (rep["N"], rep["M"], rep["kept"]) == (ref["N"], ref["J"], ref["J"] + 1)
    assert rep["pairs"] == (ref["J"] + 2) // 2
    assert rep["q_nonpos"] == ref["n_nonpos"]
    err = np.abs(out - ref["out"])
    print(f"[poly] {img.shape} N={rep['N']} J={rep['M']} max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e}",
          flush=True)
    assert err.max() <= tol


SHAPES = [(1, 1), (1, 97), (83, 1), (37, 53), (130, 257), (64, 64)]


@pytest.mark.parametrize("blur", ["iir_f32", "toeplitz_f16x2", "toeplitz_bf16x2"])
@pytest.mark.parametrize("shape", SHAPES)
def test_polynomial_small_shapes(blur, shape):
    H, W = shape
    img = gen_random(11 + H * 7 + W, H, W, "u8", "mixed")
    ss, R, sr, eps = 2.0, 6, 25.0, 1e-3
    print(f"[poly] {blur} {shape}", flush=True)
    out, rep = _run(img, _params(H, W, ss, R, sr, eps, blur))
    ref = rp.rp_shiftable_bf(img, OP[blur], ss, R, sr, eps, 255.0)
    _check(img, out, rep, ref)


@pytest.mark.parametrize("sr,eps", [(60.0, 1e-4), (30.0, 1e-3), (15.0, 1e-3), (10.0, 1e-2)])
@pytest.mark.parametrize("blur", ["iir_f32", "toeplitz_f16x2"])
def test_polynomial_sigma_r_sweep(blur, sr, eps):
    img = gen_random(3, 96, 141, "u8", "noise")
    ss, R = 3.0, 9
    print(f"[poly] {blur} sr={sr} eps={eps}", flush=True)
    out, rep = _run(img, _params(96, 141, ss, R, sr, eps, blur))
    ref = rp.rp_shiftable_bf(img, OP[blur], ss, R, sr, eps, 255.0)
    _check(img, out, rep, ref)


@pytest.mark.parametrize("R", [1, 5, 20])
def test_polynomial_box_filter(R):
    img = gen_random(21 + R, 120, 133, "u8", "mixed")
    sr, eps = 20.0, 1e-3
    print(f"[poly] box R={R}", flush=True)
    out, rep = _run(img, _params(120, 133, float(R), R, sr, eps, "toeplitz_f16x2", spatial="box"))
    ref = rp.rp_shiftable_bf(img, "box", float(R), R, sr, eps, 255.0)
    _check(img, out, rep, ref)


def test_polynomial_constant_image():
    img = np.full((70, 90), 201, np.uint8)
    out, rep = _run(img, _params(70, 90, 3.0, 9, 20.0, 1e-3, "iir_f32"))
    assert np.abs(out - 201.0).max() <= 2e-3


def test_polynomial_rectangles_workload_whole():
    """The 256x256 rectangles image (sigma_s = 3, R = 9, sigma_r = 30, global
    T = 255, eps = 1e-3) with the polynomial kernel, whole image."""
    img = config_image(1)
    for blur in ("iir_f32", "toeplitz_f16x2"):
        print(f"[poly] rect256 {blur}", flush=True)
        out, rep = _run(img, _params(256, 256, 3.0, 9, 30.0, 1e-3, blur))
        ref = rp.rp_shiftable_bf(img, OP[blur], 3.0, 9, 30.0, 1e-3, 255.0)
        _check(img, out, rep, ref)


def test_polynomial_high_order_sampled():
    """512x512 gradient image at sigma_r = 10 (N = 326 from global T = 255):
    the split-FP16 Toeplitz output at sampled pixels against eq. (BF)
    evaluated directly with the truncated polynomial kernel."""
    img = config_image(2)
    ss, R, sr, eps = 10.0, 30, 10.0, 1e-3
    out, rep = _run(img, _params(512, 512, ss, R, sr, eps, "toeplitz_f16x2"))
    tab = rp.rp_table(sr, eps, 255.0, 255.0)
    assert (rep["N"], rep["M"]) == (tab["N"], tab["J"]) and rep["N"] == 326
    rng = np.random.default_rng(2)
    ys = np.concatenate([rng.integers(0, 512, 60), [0, 511, 0, 511]])
    xs = np.concatenate([rng.integers(0, 512, 60), [0, 511, 511, 0]])
    ref = rp.rp_direct_at(img, "fir", ss, R, sr, eps, 255.0, ys, xs)
    err = np.abs(out[ys, xs] - ref)
    print(f"[poly] 512 sr=10 J={rep['M']} max={err.max():.3e}", flush=True)
    assert err.max() <= 2e-3


def test_polynomial_batch_with_raised_cosine():
    """One batch: polynomial and raised-cosine images on both blur paths; each
    grouped output equals its single-image plan."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    items = [
        (gen_random(31, 100, 120, "u8", "mixed"), _params(100, 120, 2.5, 8, 25.0, 1e-3, "iir_f32")),
        (gen_random(32, 90, 75, "u8", "mixed"), make_params(90, 75, "u8", 2.5, 25.0, 1e-3, 8, "local",
                                                            blur="iir_f32")),
        (gen_random(33, 64, 200, "u8", "mixed"), _params(64, 200, 3.0, 9, 30.0, 1e-3, "toeplitz_f16x2")),
        (gen_random(34, 120, 60, "u8", "mixed"), _params(120, 60, 4.0, 4, 20.0, 1e-3, "toeplitz_f16x2",
                                                         spatial="box")),
    ]
    xs = [torch.from_numpy(im).to("cuda") for im, _ in items]
    plan = Plan.create([p for _, p in items])
    outs, reps = plan.filter_batch(xs)
    torch.cuda.synchronize()
    plan.close()
    for (im, p), o_, r in zip(items, outs, reps):
        single, srep = _run(im, p)
        assert (r["N"], r["M"], r["pairs"]) == (srep["N"], srep["M"], srep["pairs"])
        assert np.array_equal(o_.cpu().numpy().astype(np.float64), single)
