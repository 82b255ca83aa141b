"""GPU parity: libbf.so (through its C ABI) against the FP64 oracle.

Integer results (T, N, M) must match exactly; the filtered image within
2e-3 absolute on [0, 255], scaled by range/255 for other ranges (0.514 for
16-bit images).  Max and RMS errors are printed for every case.
"""
import numpy as np
import pytest

import oracle as o
from bfsynth import CONFIGS, batch_images, config_image, gen_random

pytestmark = pytest.mark.gpu

TOL8 = 2e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(img, dtype, blur="iir_f32", **kw):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    plan = Plan.create(make_params(H, W, dtype, blur=blur, **kw))
    t = torch.from_numpy(np.ascontiguousarray(img)).to("cuda")
    out, rep = plan.filter(t)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy().astype(np.float64), rep


def run_oracle(img, dtype, sigma_s, sigma_r, eps, radius=0, t_mode="local", t_value=0.0, op="iir"):
    rng_ = 65535.0 if dtype == "u16" else 255.0
    R = radius if radius > 0 else int(np.ceil(3 * sigma_s))
    return o.algorithm2(img.astype(np.float64), op, sigma_s, R, sigma_r, eps, rng_, t_mode == "local",
                        t_value if t_value > 0 else rng_)


def compare(img, dtype, sigma_s, sigma_r, eps, radius=0, t_mode="local", t_value=0.0, label=""):
    out, rep = run_gpu(img, dtype, sigma_s=sigma_s, sigma_r=sigma_r, eps=eps, radius=radius,
                       t_mode=t_mode, t_value=t_value)
    ref = run_oracle(img, dtype, sigma_s, sigma_r, eps, radius, t_mode, t_value)
    assert rep["T"] == ref["T"], (rep, ref["T"])
    assert (rep["N"], rep["M"]) == (ref["N"], ref["M"]), (rep, ref["N"], ref["M"])
    assert rep["q_nonpos"] == ref["n_nonpos"]
    err = np.abs(out - ref["out"])
    tol = TOL8 * (65535.0 / 255.0 if dtype == "u16" else 1.0)
    print(f"[parity] {label} {img.shape} {dtype} T={rep['T']} N={rep['N']} M={rep['M']} "
          f"pairs={rep['pairs']} max={err.max():.3e} rms={np.sqrt((err ** 2).mean()):.3e} tol={tol:.3e}",
          flush=True)
    assert err.max() <= tol
    return out, rep, ref


# ------------------------------------------------------------ Algorithm 1
@pytest.mark.parametrize("shape", [(1, 1), (1, 70), (70, 1), (33, 65), (129, 300), (300, 129)])
@pytest.mark.parametrize("R", [0, 1, 2, 4, 15, 16, 30, 31, 32, 33, 40, 47, 48, 49, 200])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_dynamic_range_exact(shape, R, dtype):
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    img = gen_random(7 + shape[0] + 3 * R, *shape, dtype=dtype)
    sr = 20.0 * (257.0 if dtype == "u16" else 1.0)
    plan = Plan.create(make_params(*shape, dtype, sigma_s=2.0, sigma_r=sr, radius=R if R > 0 else 0,
                                   t_mode="local"))
    T = plan.dynamic_range(torch.from_numpy(img).to("cuda"))
    plan.close()
    Rr = R if R > 0 else 6
    assert T == o.range_T(img.astype(np.float64), Rr)


@pytest.mark.parametrize("R", [3, 16, 30, 32, 33, 40])
@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_dynamic_range_repeated_calls(R, dtype):
    """Every call on one plan starts from a clean range state: images whose T
    falls from call to call each get their own T (the one-launch tile kernel
    clears its accumulator and workgroup counter as it publishes T), and the
    filter's report agrees."""
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    H, W = 150, 170
    plan = Plan.create(make_params(H, W, dtype, sigma_s=2.0, sigma_r=20.0, radius=R, t_mode="local"))
    for seed, scale in [(11, 1.0), (12, 0.3), (13, 0.6), (14, 0.05), (15, 0.0)]:
        img = np.floor(gen_random(seed, H, W, "u8").astype(np.float64) * scale)
        img = img.astype(np.uint8 if dtype == "u8" else np.float32)
        t = torch.from_numpy(img).to("cuda")
        T = plan.dynamic_range(t)
        assert T == o.range_T(img.astype(np.float64), R), (seed, scale)
        _, rep = plan.filter(t)
        _, rep2 = plan.filter(t)
        assert rep["T"] == T and rep["flags"] == 0
        assert rep2["T"] == T and rep2["q_nonpos"] == rep["q_nonpos"]
    plan.close()


def test_dynamic_range_non_finite_values():
    """Float input with +inf, -inf and NaN: the report flags it on both range
    paths, and the next call on a clean image reports no flag."""
    torch = _torch()
    from paper_1203_5128_amd import BFError, Plan, make_params
    for R in (5, 20, 40):
        plan = Plan.create(make_params(70, 90, "f32", sigma_s=2.0, sigma_r=20.0, radius=R))
        for bad in (np.inf, -np.inf, np.nan):
            img = gen_random(83, 70, 90, "f32")
            img[33, 61] = bad
            with pytest.raises(BFError) as ei:
                plan.filter(torch.from_numpy(img).to("cuda"))
            assert ei.value.status == 5
            clean = gen_random(84, 70, 90, "f32")
            _, rep = plan.filter(torch.from_numpy(clean).to("cuda"))
            assert rep["flags"] == 0 and rep["T"] == o.range_T(clean.astype(np.float64), R)
        plan.close()


# ------------------------------------------------------- small parity sweep
SMALL = [(1, 1), (1, 17), (17, 1), (33, 65), (64, 64), (100, 257), (37, 300), (200, 33)]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_small_parity(shape, dtype):
    img = gen_random(31 * shape[0] + shape[1], *shape, dtype=dtype)
    sc = 257.0 if dtype == "u16" else 1.0
    compare(img, dtype, 2.0, 25.0 * sc, 1e-3, label="small")


@pytest.mark.parametrize("sigma_s", [0.7, 1.5, 5.0, 12.0])
@pytest.mark.parametrize("sigma_r", [8.0, 15.0, 45.0])
def test_sigma_sweep(sigma_s, sigma_r):
    img = gen_random(int(100 * sigma_s + sigma_r), 96, 130, dtype="u8")
    compare(img, "u8", sigma_s, sigma_r, 1e-3, label=f"ss={sigma_s} sr={sigma_r}")


@pytest.mark.parametrize("width", [31, 32, 33, 2047, 2049, 4100])
def test_widths_and_cross_wave_scan(width):
    img = gen_random(width, 40, width, dtype="u8")
    compare(img, "u8", 3.0, 30.0, 1e-3, label=f"W={width}")


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("width,sigma_s", [(100, 2.5), (1030, 2.5), (1040, 8.0), (1500, 2.5), (2064, 8.0),
                                           (2100, 2.5)])
def test_row_ends_inside_the_row_group(width, sigma_s, dtype):
    """Rows shorter than their row group: the horizontal pass's line ends with
    the last thread holding positions (8-bit and float; 16-bit smooths zeros
    on the threads after it).  With 16 columns per thread: W = 100 ends inside
    one 8-thread wave; W = 1030 and 1040 at the first lane of the second wave
    of a 128-thread group (1040 at the end of that lane's chunk, where the
    boundary sees the previous wave's carry at full weight); W = 1500 in the
    middle of that wave; W = 2064 at the first lane of the third wave of a
    256-thread group and W = 2100 inside it, the fourth wave all past the
    row."""
    img = gen_random(3 * width + len(dtype), 24, width, dtype=dtype)
    sc = 257.0 if dtype == "u16" else 1.0
    compare(img, dtype, sigma_s, 30.0 * sc, 1e-3, label=f"W={width} ss={sigma_s} {dtype}")


@pytest.mark.parametrize("shape", [(4097, 40), (6000, 64), (8192, 33), (24, 8192)])
def test_recursive_path_size_limits(shape):
    """Heights above 4096 take the vertical instantiation with 256 threads per
    column (one column per row group of the recursive scan); 8192 rows or
    columns is the declared limit of the recursive blur."""
    img = gen_random(shape[0] + 7 * shape[1], *shape, dtype="u8")
    compare(img, "u8", 2.0, 25.0, 1e-3, label=f"limit {shape}")


def test_global_mode_original_shiftable():
    img = gen_random(5, 80, 90, dtype="u8")
    compare(img, "u8", 3.0, 30.0, 1e-3, t_mode="global", t_value=255.0, label="global")


# ------------------------------------------------------- workload configs
def _cfg(idx):
    c = CONFIGS[idx]
    return config_image(idx), c


def test_workload1_rect256_global():
    img, c = _cfg(1)
    compare(img, "u8", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "global", c["t_value"], "cfg1")


def test_workload2_grad512_local():
    img, c = _cfg(2)
    compare(img, "u8", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "local", 0.0, "cfg2")


def test_workload3_poly2048_u16():
    img, c = _cfg(3)
    compare(img, "u16", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "local", 0.0, "cfg3")


def test_workload4_mosaic4096_iir():
    img, c = _cfg(4)
    compare(img, "f32", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "local", 0.0, "cfg4-iir")


# ------------------------------------------------------------- invariants
def test_constant_image_unchanged():
    for v, dt in ((0, "u8"), (200, "u8"), (40000, "u16"), (77.25, "f32")):
        img = np.full((50, 70), v, dtype={"u8": np.uint8, "u16": np.uint16, "f32": np.float32}[dt])
        out, rep = run_gpu(img, dt, sigma_s=3.0, sigma_r=20.0 * (257 if dt == "u16" else 1), eps=1e-3)
        assert rep["T"] == 0 and rep["N"] == 1
        assert np.abs(out - float(v)).max() <= 1e-3 * (257 if dt == "u16" else 1)


def test_affine_u8_to_u16():
    img = gen_random(77, 90, 120, "u8")
    o8, r8 = run_gpu(img, "u8", sigma_s=3.0, sigma_r=20.0, eps=1e-3)
    o16, r16 = run_gpu(img.astype(np.uint16) * 257, "u16", sigma_s=3.0, sigma_r=20.0 * 257, eps=1e-3)
    assert (r8["N"], r8["M"]) == (r16["N"], r16["M"])
    assert np.abs(o16 - 257.0 * o8).max() <= 2 * TOL8 * 257


def test_reflection_and_transpose():
    img = gen_random(78, 64, 96, "u8")
    a, _ = run_gpu(img, "u8", sigma_s=2.5, sigma_r=25.0, eps=1e-3)
    b, _ = run_gpu((255 - img).astype(np.uint8), "u8", sigma_s=2.5, sigma_r=25.0, eps=1e-3)
    c, _ = run_gpu(np.ascontiguousarray(img.T), "u8", sigma_s=2.5, sigma_r=25.0, eps=1e-3)
    assert np.abs(b - (255.0 - a)).max() <= 2 * TOL8
    assert np.abs(c - a.T).max() <= 2 * TOL8


def test_deterministic():
    img = gen_random(79, 120, 140, "u8")
    a, _ = run_gpu(img, "u8", sigma_s=4.0, sigma_r=12.0, eps=1e-3)
    b, _ = run_gpu(img, "u8", sigma_s=4.0, sigma_r=12.0, eps=1e-3)
    assert np.array_equal(a, b)


def test_pitched_buffers():
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    img = gen_random(80, 45, 70, "u8")
    big = np.zeros((45, 96), np.uint8)
    big[:, :70] = img
    plan = Plan.create(make_params(45, 70, "u8", sigma_s=2.0, sigma_r=20.0, in_pitch=96, out_pitch=80))
    tin = torch.from_numpy(big).to("cuda")
    tout = torch.full((45, 80), -7.0, device="cuda")
    with pytest.raises(ValueError):  # the whole padded buffer is not a 45 x 70 image
        plan.filter(tin, tout)
    plan.filter(tin[:, :70], tout[:, :70])
    torch.cuda.synchronize()
    plan.close()
    ref, _ = run_gpu(img, "u8", sigma_s=2.0, sigma_r=20.0, eps=1e-3)
    got = tout.cpu().numpy()
    assert np.array_equal(got[:, :70].astype(np.float64), ref)
    assert np.all(got[:, 70:] == -7.0)


def test_non_finite_input_reported():
    torch = _torch()
    from paper_1203_5128_amd import BFError, Plan, make_params
    img = gen_random(81, 20, 30, "f32")
    img[5, 7] = np.nan
    plan = Plan.create(make_params(20, 30, "f32", sigma_s=2.0, sigma_r=20.0))
    with pytest.raises(BFError) as ei:
        plan.filter(torch.from_numpy(img).to("cuda"))
    assert ei.value.status == 5
    plan.close()


def test_batch_uneven_sizes_per_image_params():
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    items = batch_images(6)
    small = [(im[:min(im.shape[0], 160), :min(im.shape[1], 200)].copy(), ss, sr) for im, ss, sr in items]
    params = [make_params(im.shape[0], im.shape[1], "u8", sigma_s=ss, sigma_r=sr, eps=1e-3) for im, ss, sr in small]
    plan = Plan.create(params)
    outs, reps = plan.filter_batch([torch.from_numpy(im).to("cuda") for im, _, _ in small])
    torch.cuda.synchronize()
    plan.close()
    for (im, ss, sr), out, rep in zip(small, outs, reps):
        ref = run_oracle(im, "u8", ss, sr, 1e-3)
        assert (rep["N"], rep["M"]) == (ref["N"], ref["M"])
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref["out"]).max()
        print(f"[parity] batch {im.shape} ss={ss:.2f} sr={sr:.2f} max={err:.3e}", flush=True)
        assert err <= TOL8


def test_graph_replays_match_eager():
    """The captured launch sequence, replayed with eager GPU work in between,
    gives bit-identical output every time and equals the direct launches."""
    import os
    torch = _torch()
    from paper_1203_5128_amd import Plan, make_params
    img = gen_random(82, 140, 170, "u8")
    t = torch.from_numpy(img).to("cuda")
    plan = Plan.create(make_params(140, 170, "u8", sigma_s=4.0, sigma_r=15.0))
    outs = []
    out = torch.empty((140, 170), device="cuda")
    for r in range(4):
        plan.filter(t, out, report=False)
        torch.cuda.synchronize()
        outs.append(out.cpu().clone())
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
    plan.close()
    os.environ["BF_GRAPH"] = "0"
    try:
        plan2 = Plan.create(make_params(140, 170, "u8", sigma_s=4.0, sigma_r=15.0))
        eager, _ = plan2.filter(t)
        torch.cuda.synchronize()
        plan2.close()
    finally:
        del os.environ["BF_GRAPH"]
    for o in outs:
        assert torch.equal(o, outs[0])
    assert torch.equal(eager.cpu(), outs[0])
