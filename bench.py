"""Benchmark of the shiftable bilateral filter on one MI355X.

One step = one call of bf_filter on the resident 512x512 8-bit workload
(gradient + step edges + noise, sigma_s = 10, sigma_r = 10, local T over the
61x61 window, eps = 1e-3, FP32 recursive Gaussian): the dynamic-range stage,
every frequency pair's blur, and the combine/divide.  The output of the timed
steps is checked against the FP64 oracle, and the oracle itself is timed on
the host cores as the CPU baseline.

Besides this plain FP32 line (`value`), the same JSON line carries the mixed
path on the same workload (split-FP16 Toeplitz blur, its error against the
oracle with the FIR operator), the batched path (64 images of uneven sizes
with per-image sigma_s, sigma_r, one grouped graph launch per step, its error
at sampled pixels against eq. (BF) evaluated directly, and the same images
filtered one by one for comparison), and the constant (box) spatial filter of
Section 4 (radius 20, sigma_r 5, eps 0.01) on the same image.

Prints one JSON line.  Only one GPU is supported: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes(stage: str, H: int, W: int, pairs: int, b_in: int, kcount: int) -> float:
    """Bytes a stage must move per launch.

    v_iir generates the four images of each pair from f and writes them
    smoothed down the columns (16 B per pixel and pair, FP32); h_combine reads
    them back and writes the output.  The range stage reads f twice and
    writes/reads the row maxima once."""
    px = H * W
    if stage == "v_iir":
        return px * (16.0 * pairs + b_in)
    if stage == "h_combine":
        return px * (16.0 * pairs + b_in + 4.0)
    if stage == "range":
        return px * 4.0 * b_in
    return 0.0


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_grad512_u8.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    return rec["traffic_bytes"] if sha.startswith(rec["source_sha256_prefix"]) else None


def cpu_baseline(img, c, mixed=None, batch=None, box=None, budget_s=25.0):
    """The CPU leg: the FP64 oracle timed on the main workload (Algorithm 2
    with the recursive operator, all host threads).  Its outputs, and the
    oracle values it computes afterwards (untimed) for the mixed line (whole
    image, FIR operator) and the batched line (sampled pixels of every image,
    each with the operator its autotuned variant uses), are the references of
    the error checks."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    f = img.astype(np.float64)
    times = []
    t_start = time.time()
    while len(times) < 3 and (time.time() - t_start) < budget_s:
        t0 = time.perf_counter()
        r = oracle.algorithm2(f, "iir", c["sigma_s"], c["radius"], c["sigma_r"], c["eps"], 255.0, True)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    base = dict(value=img.size / med / 1e6, unit="megapixels/sec", cores=threads, kind="oracle",
                sample=f"whole {img.shape[0]}x{img.shape[1]} image, Algorithm 2 end to end (FP64, IIR "
                       f"operator), median of {len(times)} runs, {med:.2f} s each")
    refs = dict(iir=r)
    if mixed is not None:
        refs["fir"] = oracle.algorithm2(f, "fir", c["sigma_s"], c["radius"], c["sigma_r"], c["eps"], 255.0, True)
    if batch is not None:
        vals = []
        for (im, ss, sr), rep, (ys, xs) in batch:
            g = im.astype(np.float64)
            R = int(np.ceil(3 * ss))
            if rep["variant"] == "iir_f32":  # no pointwise form of the recursive operator: whole image
                vals.append(oracle.algorithm2(g, "iir", ss, R, sr, 1e-3, 255.0, True)["out"][ys, xs])
            else:
                vals.append(oracle.direct_fir_at(g, ss, R, rep["N"], rep["M"], sr, ys, xs))
        refs["batch"] = vals
    if box is not None:  # eq. (BF) directly with the box filter at the sampled pixels
        ys, xs = box
        R, sr, eps = BOX["radius"], BOX["sigma_r"], BOX["eps"]
        T = oracle.range_T(f, R)
        N = oracle.order(T, sr)
        M = oracle.trunc_rule(N, sr, eps)
        refs["box"] = dict(T=T, N=N, M=M, vals=oracle.direct_box_at(f, R, N, M, sr, ys, xs))
    return refs, base


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def mixed_line(img, c, x, steps, warmup):
    """The split-FP16 Toeplitz path on the same workload; returns the line
    and the output (host) for the error check."""
    import torch
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    out = torch.empty((H, W), dtype=torch.float32, device=x.device)
    plan = Plan.create(make_params(H, W, "u8", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "local",
                                   blur="toeplitz_f16x2"))
    _, rep = plan.filter(x, out, report=True)
    sec = time_steps(lambda: plan.filter(x, out, report=False), steps, warmup)
    plan.close()
    line = dict(blur="toeplitz_f16x2", value=round(H * W / sec / 1e6, 3), unit="megapixels/sec",
                ms_per_step=round(sec * 1e3, 5), dtype="f16 hi+lo operands, f32 accumulation",
                N=rep["N"], M=rep["M"])
    return line, out.cpu().numpy().astype(np.float64)


BOX = dict(radius=20, sigma_r=5.0, eps=1e-2)  # the paper's box setting (Section 4)


def box_line(img, x, steps, warmup):
    """The constant (box) spatial filter of radius 20 with sigma_r = 5 and
    eps = 0.01 on the same image (split-FP16 Toeplitz kernels, unit taps);
    returns the line and the output at sampled pixels for the error check."""
    import torch
    from paper_1203_5128_amd import Plan, make_params
    H, W = img.shape
    out = torch.empty((H, W), dtype=torch.float32, device=x.device)
    plan = Plan.create(make_params(H, W, "u8", float(BOX["radius"]), BOX["sigma_r"], BOX["eps"], BOX["radius"],
                                   "local", blur="toeplitz_f16x2", spatial="box"))
    _, rep = plan.filter(x, out, report=True)
    sec = time_steps(lambda: plan.filter(x, out, report=False), steps, warmup)
    plan.close()
    line = dict(spatial="box", blur="toeplitz_f16x2", radius=BOX["radius"], sigma_r=BOX["sigma_r"],
                eps=BOX["eps"], value=round(H * W / sec / 1e6, 3), unit="megapixels/sec",
                ms_per_step=round(sec * 1e3, 5), T=rep["T"], N=rep["N"], M=rep["M"], pairs=rep["pairs"])
    rng = np.random.default_rng(9)
    ys = np.concatenate([rng.integers(0, H, 150), [0, H - 1, 0, H - 1]])
    xs = np.concatenate([rng.integers(0, W, 150), [0, W - 1, W - 1, 0]])
    return line, (ys, xs, out.cpu().numpy()[ys, xs].astype(np.float64))


def sequential_batch(steps, warmup):
    """The 64 images of the batch workload filtered one after another, each
    by its own single-image plan (recursive blur): the reference for what the
    grouped batch launch gains."""
    import torch
    from bfsynth import batch_images
    from paper_1203_5128_amd import Plan, make_params
    items = batch_images()
    xs = [torch.from_numpy(im).to("cuda:0") for im, _, _ in items]
    outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in xs]
    plans = [Plan.create(make_params(im.shape[0], im.shape[1], "u8", sigma_s=ss, sigma_r=sr, eps=1e-3,
                                     blur="iir_f32")) for im, ss, sr in items]

    def step():
        for pl, x, o in zip(plans, xs, outs):
            pl.filter(x, o, report=False)
    sec = time_steps(step, steps, warmup)
    for pl in plans:
        pl.close()
    px = sum(im.size for im, _, _ in items)
    return dict(blur="iir_f32", images=len(items), value=round(px / sec / 1e6, 3), unit="megapixels/sec",
                ms_per_step=round(sec * 1e3, 5)), [o.cpu() for o in outs]


def batched_line(blur, steps, warmup):
    """The 64-image workload (uneven sizes, per-image sigma_s, sigma_r) with
    every image on `blur` ("auto": each image's autotuned variant); returns
    the line and (item, report, sampled pixels, sampled outputs) of the
    images whose outputs are checked (all for the FIR variants, every fourth
    for the recursive one, whose oracle runs on the whole image)."""
    import torch
    from bfsynth import batch_images
    from paper_1203_5128_amd import Plan, make_params
    items = batch_images()
    xs = [torch.from_numpy(im).to("cuda:0") for im, _, _ in items]
    outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in xs]
    t0 = time.perf_counter()
    plan = Plan.create([make_params(im.shape[0], im.shape[1], "u8", sigma_s=ss, sigma_r=sr, eps=1e-3, blur=blur)
                        for im, ss, sr in items])
    plan_s = time.perf_counter() - t0
    _, reps = plan.filter_batch(xs, outs, report=True)
    sec = time_steps(lambda: plan.filter_batch(xs, outs, report=False), steps, warmup)
    plan.close()
    px = sum(im.size for im, _, _ in items)
    chosen = {}
    for r in reps:
        chosen[r["variant"]] = chosen.get(r["variant"], 0) + 1
    line = dict(blur=blur, images=len(items), megapixels=round(px / 1e6, 3), value=round(px / sec / 1e6, 3),
                unit="megapixels/sec", ms_per_step=round(sec * 1e3, 5), variants=chosen,
                plan_s=round(plan_s, 2))
    rng = np.random.default_rng(5)
    samples = []
    for i, (it, out, r) in enumerate(zip(items, outs, reps)):
        if r["variant"] == "iir_f32" and i % 4:
            continue
        ys, xs_ = rng.integers(0, it[0].shape[0], 12), rng.integers(0, it[0].shape[1], 12)
        samples.append((it, r, (ys, xs_), out.cpu().numpy()[ys, xs_].astype(np.float64)))
    return line, samples


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="plain FP32 line only (no mixed/batched lines)")
    ap.add_argument("--lines", default="mixed,batch,box",
                    help="extra lines besides the plain one: any of mixed, batch, box (empty: none)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB mebibytes (a kernel of known "
                         "traffic against which the HBM byte counters are scaled)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (--gpus {args.gpus} requested); "
              "multi-GPU sharding is a design note only", file=sys.stderr)
        sys.exit(2)

    import torch
    from bfsynth import CONFIGS, config_image
    from paper_1203_5128_amd import Plan, make_params

    if args.copy_calibration:
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    c = CONFIGS[2]
    img = config_image(2)
    H, W = img.shape
    dev = torch.device("cuda:0")
    x = torch.from_numpy(img).to(dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    plan = Plan.create(make_params(H, W, "u8", c["sigma_s"], c["sigma_r"], c["eps"], c["radius"], "local",
                                   blur="iir_f32"))
    stream = torch.cuda.current_stream()

    _, rep = plan.filter(x, out, stream=stream, report=True)
    for _ in range(args.warmup):
        plan.filter(x, out, stream=stream, report=False)
    torch.cuda.synchronize()

    # timed region: the captured launch sequence replayed, nothing else
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.filter(x, out, stream=stream, report=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = H * W * args.steps / (t1 - t0) / 1e6

    # per-stage device time: the same steps launched directly with HIP events
    # between the stages on the launch stream
    plan.profile(True)
    plan.profile_read()
    for _ in range(args.steps):
        plan.filter(x, out, stream=stream, report=False)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)

    # the dominant kernel and its roofline
    pairs = rep["pairs"]
    b_in = 1
    dom = max(prof, key=lambda s: prof[s][0])
    dom_ms, dom_n = prof[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    bytes_launch = algorithmic_bytes(dom, H, W, pairs, b_in, pairs)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    stages = {s: dict(ms_per_step=v[0] / args.steps, launches_per_step=v[1] / args.steps)
              for s, v in prof.items() if v[1]}

    result = dict(metric="megapixels/sec of shiftable BF at max err <=2e-3 (plain FP32 vs mixed/batched)",
                  value=round(value, 3), unit="megapixels/sec", n_gpus=1, steps=args.steps, warmup=args.warmup,
                  ms_per_step=round(ms_step, 5), higher_is_better=True, scaling="weak", vs_baseline=None,
                  dtype="f32", data="synthetic",
                  config=dict(workload="grad512_u8_local", H=H, W=W, input="u8", sigma_s=c["sigma_s"],
                              radius=c["radius"], sigma_r=c["sigma_r"], eps=c["eps"], t_mode="local",
                              blur="iir_f32", T=rep["T"], N=rep["N"], M=rep["M"], pairs=pairs),
                  roofline=dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                                avg_launch_ms=round(avg_ms, 5), bytes_per_launch=bytes_launch,
                                traffic=measured_traffic(dom)),
                  stages=stages)

    got = out.cpu().numpy().astype(np.float64)
    plan.close()
    mixed = None
    batches = {}
    lines = set() if args.no_extra else {t for t in args.lines.split(",") if t}
    if "mixed" in lines:
        mixed, mixed_out = mixed_line(img, c, x, args.steps, args.warmup)
        result["mixed"] = mixed
    if "batch" in lines:
        bsteps = max(3, args.steps // 20)
        for key, blur in (("plain", "iir_f32"), ("mixed", "toeplitz_f16x2"), ("auto", "auto")):
            batches[key] = batched_line(blur, bsteps, 2)
        result["batched"] = dict(workload="batch64_u8_local", **{k: v[0] for k, v in batches.items()})
        result["batched"]["speedup_mixed_vs_plain"] = round(
            batches["mixed"][0]["value"] / batches["plain"][0]["value"], 3)
        result["batched"]["speedup_auto_vs_plain"] = round(
            batches["auto"][0]["value"] / batches["plain"][0]["value"], 3)
        seq, seq_outs = sequential_batch(max(2, bsteps // 4), 1)
        result["batched"]["sequential"] = seq
        result["batched"]["speedup_batched_vs_sequential"] = round(batches["plain"][0]["value"] / seq["value"], 3)
    box = None
    if "box" in lines:
        box, box_out = box_line(img, x, args.steps, args.warmup)
        result["box"] = box
    # accuracy of the timed outputs against the FP64 oracle (the CPU leg)
    if not args.no_cpu_baseline:
        samples = [smp for v in batches.values() for smp in v[1]]
        refs, cpu = cpu_baseline(img, c, mixed=mixed, batch=[(it, r, p) for it, r, p, _ in samples] or None,
                                 box=(box_out[0], box_out[1]) if box is not None else None)
        ref = refs["iir"]
        err = np.abs(got - ref["out"])
        result["max_err"] = float(err.max())
        result["rms_err"] = float(np.sqrt((err ** 2).mean()))
        result["err_ok"] = bool(err.max() <= 2e-3 and (ref["N"], ref["M"]) == (rep["N"], rep["M"]))
        result["cpu_baseline"] = cpu
        if mixed is not None:
            e2 = np.abs(mixed_out - refs["fir"]["out"])
            mixed.update(max_err=float(e2.max()), rms_err=float(np.sqrt((e2 ** 2).mean())),
                         err_ok=bool(e2.max() <= 2e-3 and (refs["fir"]["N"], refs["fir"]["M"]) == (mixed["N"], mixed["M"])))
        if batches:
            errs = [float(np.abs(v - r).max()) for (_, _, _, v), r in zip(samples, refs["batch"])]
            i0 = 0
            for key, (line, smp) in batches.items():
                worst = max(errs[i0:i0 + len(smp)])
                i0 += len(smp)
                line.update(sampled_max_err=worst, err_ok=bool(worst <= 2e-3))
        if box is not None:
            rb = refs["box"]
            e3 = np.abs(box_out[2] - rb["vals"])
            box.update(sampled_max_err=float(e3.max()),
                       err_ok=bool(e3.max() <= 2e-3 and (rb["T"], rb["N"], rb["M"]) == (box["T"], box["N"], box["M"])))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
