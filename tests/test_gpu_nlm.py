"""GPU parity of the shiftable non-local means (eqs. (NL1), (NL2)) against
the FP64 oracle's direct sums with the same truncated product kernel
(oracle/nlm.py): patch sizes 2..4 with several offset sets, small and ragged
shapes, the box window of eq. (NL1) and the sampled Gaussian weights, both
split Toeplitz variants, local and global T, and the 256x256 rectangles
image with a three-sample patch over an 11x11 window (1099 frequency
multi-indices), whole image."""
import numpy as np
import pytest

from bfsynth import config_image, gen_random
from oracle import nlm

pytestmark = pytest.mark.gpu

P2 = [(0, 0), (0, 1)]
P3 = [(0, 0), (0, 1), (1, 0)]
P4 = [(0, 0), (0, -1), (-1, 0), (2, 2)]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(img, patch, ss, R, sr, eps, blur="toeplitz_f16x2", spatial="box", t_mode="local", t_value=0.0):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    plan = Plan.create(make_params(H, W, "u8", sigma_s=ss, sigma_r=sr, eps=eps, radius=R, t_mode=t_mode,
                                   t_value=t_value, blur=blur, spatial=spatial, patch=patch))
    out, rep = plan.filter(torch.from_numpy(np.ascontiguousarray(img)).to("cuda"))
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().astype(np.float64), rep


def _check(img, patch, op, ss, R, sr, eps, out, rep, t_local=True, t_value=0.0, tol=2e-3):
    ref = nlm.nlm_algorithm(img, patch, op, ss, R, sr, eps, 255.0, t_local, t_value)
    assert (rep["T"], rep["N"], rep["M"]) == (ref["T"], ref["N"], ref["M"])
    assert rep["pairs"] == ref["pairs"]
    assert rep["q_nonpos"] == ref["n_nonpos"]
    err = np.abs(out - ref["out"])
    print(f"[nlm] {img.shape} p={len(patch)} {op} N={rep['N']} M={rep['M']} pairs={rep['pairs']} "
          f"max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e}", flush=True)
    assert err.max() <= tol


@pytest.mark.parametrize("blur", ["toeplitz_f16x2", "toeplitz_bf16x2"])
@pytest.mark.parametrize("patch", [P2, P3, P4])
@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (29, 1), (37, 53), (70, 131)])
def test_nlm_shapes_and_patches(shape, patch, blur):
    H, W = shape
    img = gen_random(100 + 3 * H + W, H, W, "u8", "mixed")
    R, sr, eps = 3, 45.0, 1e-3
    print(f"[nlm] {blur} {shape} p={len(patch)}", flush=True)
    out, rep = _run(img, patch, 1.0, R, sr, eps, blur)
    _check(img, patch, "box", 1.0, R, sr, eps, out, rep)


@pytest.mark.parametrize("sr,eps", [(60.0, 1e-3), (30.0, 1e-2), (40.0, 1e-4)])
def test_nlm_sigma_r_and_eps(sr, eps):
    img = gen_random(7, 64, 90, "u8", "noise")
    R = 4
    print(f"[nlm] sr={sr} eps={eps}", flush=True)
    out, rep = _run(img, P3, 1.0, R, sr, eps)
    _check(img, P3, "box", 1.0, R, sr, eps, out, rep)


def test_nlm_gaussian_window_weights():
    img = gen_random(8, 80, 75, "u8", "mixed")
    ss, R, sr, eps = 2.0, 6, 40.0, 1e-3
    out, rep = _run(img, P3, ss, R, sr, eps, spatial="gaussian_fir")
    _check(img, P3, "fir", ss, R, sr, eps, out, rep)


def test_nlm_global_T():
    img = gen_random(9, 60, 61, "u8", "mixed")
    R, sr, eps = 3, 50.0, 1e-3
    out, rep = _run(img, P2, 1.0, R, sr, eps, t_mode="global", t_value=255.0)
    _check(img, P2, "box", 1.0, R, sr, eps, out, rep, t_local=False, t_value=255.0)


def test_nlm_constant_image():
    img = np.full((50, 70), 90, np.uint8)
    out, rep = _run(img, P4, 1.0, 3, 40.0, 1e-3)
    assert rep["T"] == 0.0
    assert np.abs(out - 90.0).max() <= 2e-3


def test_nlm_rectangles_workload_whole():
    """The 256x256 rectangles image, patch (0,0), (0,1), (1,0), 11x11 box
    window, sigma_r = 40, eps = 1e-3, local T: whole image."""
    img = config_image(1)
    R, sr, eps = 5, 40.0, 1e-3
    for blur in ("toeplitz_f16x2", "toeplitz_bf16x2"):
        print(f"[nlm] rect256 {blur}", flush=True)
        out, rep = _run(img, P3, 1.0, R, sr, eps, blur)
        _check(img, P3, "box", 1.0, R, sr, eps, out, rep)
