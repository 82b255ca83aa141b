"""GPU parity on an image built so that the denominator (f2) is negative.

The truncated kernel phi_eps of eq. (approx) may dip down to -eps (Section 3).
On a flat background with isolated pixels 140 levels darker, at sigma_r = 25,
eps = 0.05 and the global T = 255, phi_eps(140) is about -0.021 and every
isolated pixel's denominator is negative; everywhere else it is positive.
The library must count the same pixels as the FP64 oracle and return the
input there (the fallback), on the recursive and on the Toeplitz blur, for
8-bit, 16-bit (intensities and sigma_r scaled by 257) and float input.
"""
import numpy as np
import pytest

import oracle as o

pytestmark = pytest.mark.gpu


def _image(H=100, W=131, bg=200.0, spot=60.0):
    f = np.full((H, W), bg)
    ys, xs = np.meshgrid(np.arange(10, H, 32), np.arange(12, W, 33), indexing="ij")
    f[ys, xs] = spot
    return f, ys.ravel(), xs.ravel()


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("blur,op", [("iir_f32", "iir"), ("toeplitz_f16x2", "fir"), ("toeplitz_bf16x2", "fir")])
def test_negative_denominator_fallback(blur, op, dtype):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1203_5128_amd import Plan, make_params
    f, ys, xs = _image()
    sc = 257.0 if dtype == "u16" else 1.0
    rng_ = 255.0 * sc
    img = (f * sc).astype({"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[dtype])
    ss, R, sr, eps = 6.0, 18, 25.0 * sc, 0.05
    ref = o.algorithm2(img.astype(np.float64), op, ss, R, sr, eps, rng_, False, rng_)
    assert ref["n_nonpos"] == len(ys) == 12
    H, W = img.shape
    plan = Plan.create(make_params(H, W, dtype, sigma_s=ss, sigma_r=sr, eps=eps, radius=R,
                                   t_mode="global", t_value=rng_, blur=blur))
    print(f"[qneg] {blur} {dtype} {img.shape}", flush=True)
    out, rep = plan.filter(torch.from_numpy(img).to("cuda"))
    torch.cuda.synchronize()
    plan.close()
    got = out.cpu().numpy().astype(np.float64)
    assert (rep["N"], rep["M"]) == (ref["N"], ref["M"]) == (42, 15)
    assert rep["q_nonpos"] == ref["n_nonpos"]
    assert np.array_equal(got[ys, xs], img[ys, xs].astype(np.float64))
    err = np.abs(got - ref["out"])
    print(f"[qneg] max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e}", flush=True)
    assert err.max() <= 2e-3 * sc
