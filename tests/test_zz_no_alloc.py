"""bf_filter_noalloc through the C ABI: the same kernels and tables as
bf_filter, with the working memory in the library's static per-device array.

Two calls in a row on one device, the second with a smaller image (the array
keeps the first call's contents, so the second checks that the state it needs
cleared is cleared), each compared with bf_filter on the same plan: the same
launch shape gives the same bits; an image whose pairs need several launches
in the 256 MiB differs from bf_filter's one launch only in the order its pair
sums are added, within the 2e-3 bar (scaled by 257 for 16-bit images).
"""
import ctypes

import numpy as np
import pytest

from bfsynth import config_image, gen_random

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(plan, img, torch):
    """bf_filter, then bf_filter_noalloc, on the same plan and input."""
    d = torch.from_numpy(img).to("cuda")
    ref, rep_ref = plan.filter(d)
    out = torch.full(img.shape, -1.0, dtype=torch.float32, device="cuda")
    out, rep = plan.filter_noalloc(d, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), rep_ref, out.cpu().numpy(), rep


def _same_report(a, b):
    for k in ("T", "T_used", "N", "M", "kept", "pairs", "variant", "flags", "q_nonpos"):
        assert a[k] == b[k], (k, a[k], b[k])


def test_noalloc_two_calls_second_smaller():
    torch = _cuda()
    from paper_1203_5128_amd import Plan, make_params
    # first call: the 512x512 8-bit workload on the recursive blur (all its
    # pairs fit one launch in the static array, as in bf_filter)
    a = config_image(2)
    pa = Plan.create(make_params(512, 512, "u8", sigma_s=10.0, sigma_r=10.0, eps=1e-3, radius=30,
                                 t_mode="local", blur="iir_f32"))
    print("[noalloc] call 1: 512x512 u8 iir_f32 local T", flush=True)
    ref, rep_ref, got, rep = _both(pa, a, torch)
    pa.close()
    _same_report(rep_ref, rep)
    assert rep["T"] == 212.0 and rep["pairs"] == 39
    assert np.array_equal(got, ref)
    # second call: a smaller 16-bit image with a smaller T on the Toeplitz blur
    b = gen_random(77, 100, 131, "u16", "mixed") // 4
    pb = Plan.create(make_params(100, 131, "u16", sigma_s=3.0, sigma_r=2000.0, eps=1e-3, radius=9,
                                 t_mode="local", blur="toeplitz_f16x2"))
    print("[noalloc] call 2: 100x131 u16 toeplitz_f16x2 local T", flush=True)
    ref, rep_ref, got, rep = _both(pb, b, torch)
    pb.close()
    _same_report(rep_ref, rep)
    assert rep["T"] < 65535.0 / 4 + 1
    assert np.array_equal(got, ref)


def test_noalloc_several_launches():
    """2048x2048 16-bit workload: one pair's smoothed images take 64 MiB, so
    the static array holds three pairs per launch where bf_filter runs all of
    them in one."""
    torch = _cuda()
    from paper_1203_5128_amd import Plan, make_params
    f = config_image(3)
    p = Plan.create(make_params(2048, 2048, "u16", sigma_s=8.0, sigma_r=800.0, eps=1e-4, radius=24,
                                t_mode="local", blur="iir_f32"))
    print("[noalloc] 2048x2048 u16 iir_f32 local T", flush=True)
    ref, rep_ref, got, rep = _both(p, f, torch)
    p.close()
    _same_report(rep_ref, rep)
    err = np.abs(got.astype(np.float64) - ref)
    print(f"[noalloc] pairs={rep['pairs']} max diff vs bf_filter {err.max():.3e}", flush=True)
    assert err.max() <= 2e-3 * 257


def test_noalloc_rejects_images_beyond_the_array():
    """A 4096x4096 image on the recursive blur needs 256 MiB of smoothed
    images for a single pair, more than the array: refused before any launch,
    and the output is untouched."""
    torch = _cuda()
    from paper_1203_5128_amd import bf, Plan, make_params
    p = Plan.create(make_params(4096, 4096, "u8", sigma_s=2.0, sigma_r=100.0, eps=1e-3, radius=6,
                                t_mode="global", blur="iir_f32"))
    img = torch.zeros((4096, 4096), dtype=torch.uint8, device="cuda")
    out = torch.full((4096, 4096), 7.0, dtype=torch.float32, device="cuda")
    st = bf.lib().bf_filter_noalloc(p.handle, img.data_ptr(), out.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream, None)
    torch.cuda.synchronize()
    assert st == bf.BF_ERR_UNSUPPORTED
    assert "MiB" in bf.bf_last_error_detail()
    assert bool((out == 7.0).all())
    assert bf.lib().bf_filter_noalloc(None, img.data_ptr(), out.data_ptr(), None, None) == bf.BF_ERR_INVALID_ARG
    p.close()


def test_noalloc_polynomial_kernel_and_nlm():
    """The polynomial-kernel tables and the non-local-means patch words go
    through the same static working memory.  The polynomial plans fit one
    launch (equal to bf_filter bit for bit); the non-local-means plan's up to
    1372 multi-index pairs need about 460 MB of smoothed images, so the
    static array runs them in two launches and only the order of the pair
    sums differs (within the 2e-3 bar)."""
    torch = _cuda()
    from paper_1203_5128_amd import Plan, make_params
    img = gen_random(91, 120, 170, "u8", "mixed")
    cases = [
        ("poly iir", make_params(120, 170, "u8", sigma_s=3.0, sigma_r=25.0, eps=1e-3, radius=9, t_mode="global",
                                 blur="iir_f32", range_kernel="polynomial")),
        ("poly toeplitz", make_params(120, 170, "u8", sigma_s=3.0, sigma_r=25.0, eps=1e-3, radius=9,
                                      t_mode="global", blur="toeplitz_f16x2", range_kernel="polynomial")),
        ("nlm", make_params(120, 170, "u8", sigma_s=1.0, sigma_r=45.0, eps=1e-3, radius=3, t_mode="local",
                            blur="toeplitz_f16x2", spatial="box", patch=[(0, 0), (0, 1), (1, 0)])),
    ]
    for name, p in cases:
        plan = Plan.create(p)
        print(f"[noalloc] {name}", flush=True)
        ref, rep_ref, got, rep = _both(plan, img, torch)
        plan.close()
        _same_report(rep_ref, rep)
        if name == "nlm":
            assert np.abs(got.astype(np.float64) - ref).max() <= 2e-3
        else:
            assert np.array_equal(got, ref), name
