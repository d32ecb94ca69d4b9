#!/usr/bin/env python
"""Throughput of the Fourier local Laplacian filter on one MI355X.

Workload: one 3840x2160 RGB synthetic image (channels filtered independently),
8 pyramid levels, K = 8 Fourier terms, sigma_r = 0.1, detail boost m = 3.
A step is one complete filter of that image (fit, all 2K+1 pyramids, the
per-level product-sum and the collapse) with the input already resident in HBM.
The headline value uses float32 pyramid storage; the float16- and
bfloat16-storage forms are reported beside it.

Prints ONE JSON line on stdout.  Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_uhd_rgb_k8.txt")


def kernel_source_digest():
    """sha256 over the native sources (kernels and launch configuration)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2206_04681_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".h", ".hip", ".cpp")):
            h.update(fn.encode())
            h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when it is absent or was taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_digest():
        return None
    v = kv.get(f"{kernel}_hbm_bytes_per_launch")
    return float(v) if v else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def kernel_profile(torch, ctx, fn, steps):
    ctx.timing(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    rows = ctx.timing_read()
    ctx.timing(False)
    for r in rows:
        r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
        r["gbs"] = r["bytes"] / (r["total_ms"] * 1e-3) / 1e9 if r["total_ms"] > 0 else 0.0
    return rows


def run_form(torch, fllf, storage, x, w, steps, warmup):
    ctx = fllf.FourierLLF(storage)
    out = torch.empty_like(x)
    fj, _ = ctx._prepare(fllf.Job(x, w.levels, w.sigma_r, w.m, w.K, out=out))
    ws = ctx.workspace(ctx.workspace_size([fj]))
    stream = torch.cuda.current_stream()

    def step():
        ctx.run_jobs([fj], workspace=ws, stream=stream)

    ms = time_steps(torch, step, steps, warmup)
    log(f"{storage}: {ms:.4f} ms/step")
    prof = kernel_profile(torch, ctx, step, steps)
    per_step_bytes = sum(r["bytes"] for r in prof) / steps
    return dict(ms=ms, kernels=prof, alg_bytes_per_step=per_step_bytes, ctx=ctx, out=out)


def cpu_baseline(w):
    """FP64 oracle on a bounded sample: channel 0 of the workload image (one of
    its three channels), same levels/K/sigma_r/m; single process."""
    import numpy as np
    from oracle import fourier_llf_ref as ref
    from paper_2206_04681_amd.synth import synth_image
    img = synth_image(w.height, w.width, 1, seed=w.seed, n_rect=w.n_rect, n_disk=w.n_disk, noise=w.noise)
    crop = img[0].astype(np.float64)
    t0 = time.perf_counter()
    ref.fourier_llf(crop, w.levels, w.sigma_r, w.m, w.K)
    dt = time.perf_counter() - t0
    chan_mpix = crop.size / 1e6
    # one RGB image pixel = 3 channel pixels
    return dict(value=round(chan_mpix / 3.0 / dt, 4), unit="MPix/s", cores=1, kind="oracle",
                sample=f"channel 0 of the 3840x2160 workload image "
                       f"({chan_mpix:.2f} channel-MPix = {chan_mpix / 3:.2f} RGB-MPix), "
                       f"FP64 NumPy oracle, single process, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="f32,f16,bf16")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy a buffer of this many bytes 3 times (counter calibration)")
    ap.add_argument("--digest", action="store_true", help="print the kernel source digest and exit")
    args = ap.parse_args()
    if args.digest:
        print(kernel_source_digest())
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not part of it "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 3}), flush=True)
        return
    from paper_2206_04681_amd import fllf
    from paper_2206_04681_amd.synth import UHD_RGB as w

    fllf.lib()
    log("generating the 3840x2160 RGB synthetic image")
    x = torch.from_numpy(w.image()).cuda()
    torch.cuda.synchronize()
    forms = {}
    for storage in args.forms.split(","):
        forms[storage] = run_form(torch, fllf, storage, x, w, args.steps, args.warmup)

    main_key = args.forms.split(",")[0]  # f32 unless a run selects other forms
    main_form = forms[main_key]
    ms = main_form["ms"]
    mpix = w.height * w.width / 1e6
    dom = main_form["kernels"][0]
    dom_avg_s = dom["total_ms"] * 1e-3 / dom["launches"]
    dom_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_bytes / dom_avg_s / 1e9
    result = {
        "metric": "MPix/s Fourier LLF 4K RGB K=8 (FP32 vs FP16-store); p50/p99 serve latency",
        "value": round(mpix / (ms * 1e-3), 2),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fourier_llf_3840x2160_rgb", "width": w.width, "height": w.height,
                   "channels": w.channels, "levels": w.levels, "K": w.K, "sigma_r": w.sigma_r,
                   "m": w.m, "pyramid_storage": main_key},
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom["name"]), "avg_launch_us": round(dom_avg_s * 1e6, 2),
                     "alg_bytes_per_launch": int(dom_bytes)},
        "step_alg_gbs": round(main_form["alg_bytes_per_step"] / (ms * 1e-3) / 1e9, 1),
        "kernels": {k: [dict(name=r["name"], launches=r["launches"] // args.steps,
                             avg_us=round(r["avg_us"], 2), gbs=round(r["gbs"], 1))
                        for r in f["kernels"]] for k, f in forms.items()},
    }
    for k, f in forms.items():
        if k != main_key:
            result[f"{k}_store"] = {"value": round(mpix / (f["ms"] * 1e-3), 2), "unit": "MPix/s",
                                    "ms_per_step": round(f["ms"], 5),
                                    "speedup_vs_f32": round(ms / f["ms"], 3)}
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
