#!/usr/bin/env python3
"""Throughput of Noise2Fast denoising on one MI355X.

Workload: 512x512 grayscale images (blobs scene, seed 0) with Gaussian noise
sigma 15, 25 and 50 (/255, noise seeds 1, 2, 3), each trained from scratch
with the paper's early-stopping rule (patience 100) and returned as the
mean of the last 100 validation outputs.  One "step" denoises one image to
convergence (standardise, checkerboard downsample, train, validate every
epoch, stop, write the output); steps cycle through the three noise levels.
The inputs sit in HBM before the timed region starts.

Prints one JSON line: images/s (and Mpx/s, per-image latency and PSNR), the
roofline position of the dominant convolution kernel measured with HIP
events over the timed region, and the CPU FP64 oracle timed on a bounded
sample of the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK = {"fp32": 157.3, "bf16": 2500.0}      # dense MFMA TFLOP/s, MI355X
CONV_FLOP_PER_PX = 2 * 9 * 64 * 64          # one 64->64 3x3 conv pass per pixel
KNAMES = {0: "conv3x3_fwd", 1: "conv3x3_bwd_data", 2: "conv3x3_wgrad"}


def cpu_baseline(noisy, epochs_per_image, sample_steps: int = 1):
    """Time the FP64 oracle on `sample_steps` training steps plus one
    validation of one 512x512 image, and extrapolate to whole images with
    the GPU run's epochs to convergence."""
    import numpy as np
    from oracle import n2f_oracle as O
    from paper_2108_10209_amd import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    h = O.Hyper()
    xs, _, _ = O.standardize(noisy)
    pairs = O.training_pairs(xs)
    st = O.new_state(synth.init_params(1, 0)[0])
    t0 = time.perf_counter()
    for i in range(sample_steps):
        inp, tgt = pairs[i % 4]
        st, _, _, _ = O.train_step(st, 1, inp, tgt[0], h)
    t_step = (time.perf_counter() - t0) / sample_steps
    t0 = time.perf_counter()
    O.validate(st.theta, 1, xs, 0, h)
    t_val = time.perf_counter() - t0
    sec_epoch = 4 * t_step + t_val
    sec_image = sec_epoch * epochs_per_image
    return {"value": 1.0 / sec_image, "unit": "images/s", "cores": int(cores), "kind": "oracle",
            "sec_per_epoch": sec_epoch,
            "sample": f"{sample_steps} training step(s) + 1 validation of the 512x512 sigma=25 image "
                      f"({sample_steps * t_step + t_val:.1f} s), extrapolated x {epochs_per_image:.0f} epochs "
                      f"(mean epochs to convergence of the GPU run)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32")
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--max-epochs", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time one launch in N of each conv kernel class with HIP events")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device (a plain copy of known size, to scale HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): each image is an independent run, "
              "so several GPUs would each take their own images with no communication.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth

    dev = torch.device("cuda:0")
    sigmas = [15, 25, 50]
    imgs = []
    for i, s in enumerate(sigmas):
        clean, noisy = synth.single_512(s, noise_seed=i + 1, size=args.size)
        imgs.append((s, clean, noisy, torch.from_numpy(noisy).to(dev)))
    prec = n2f.BF16 if args.precision == "bf16" else n2f.FP32
    cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs)
    ws = torch.empty(n2f.workspace_bytes(args.size, args.size, 1, cfg), dtype=torch.uint8, device=dev)

    def step(i):
        s, clean, noisy, x = imgs[i % len(imgs)]
        t0 = time.perf_counter()
        run = n2f.Run(x, cfg, ws=ws)
        _, status = run.run_epochs(0, args.max_epochs)
        y = run.result()
        torch.cuda.synchronize()
        lat = time.perf_counter() - t0
        e, be, _, _ = run.progress(0)
        run.close()
        return y, e, be, lat, status

    for i in range(args.warmup):
        step(i)
        print(f"warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    n2f.profile_begin(args.profile_every)
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step(i))
        print(f"step {i} done: {outs[-1][1]} epochs, {outs[-1][3]:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n2f.profile_end()

    psnrs, epochs, lats = [], [], []
    for i, (y, e, be, lat, status) in enumerate(outs):
        s, clean, noisy, _ = imgs[i % len(imgs)]
        psnrs.append({"sigma": s, "psnr": round(synth.psnr(y.cpu().numpy(), clean), 3),
                      "noisy_psnr": round(synth.psnr(noisy, clean), 3), "epochs": e, "best_epoch": be,
                      "capped": status == n2f.WCAPPED})
        epochs.append(e)
        lats.append(lat)

    prof = {c: n2f.profile_read(c) for c in KNAMES}
    dom = max(prof, key=lambda c: prof[c][0])
    ms, nl, px = prof[dom]
    achieved = px * CONV_FLOP_PER_PX / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    kern = {KNAMES[c]: {"total_ms": round(prof[c][0], 3), "launches": prof[c][1],
                        "avg_us": round(1e3 * prof[c][0] / max(prof[c][1], 1), 2),
                        "tflops": round(prof[c][2] * CONV_FLOP_PER_PX / max(prof[c][0], 1e-9) / 1e9, 2)}
            for c in KNAMES}

    ips = args.steps / wall
    npx = args.size * args.size
    result = {
        "metric": "images/s denoised to convergence (512x512 grayscale, sigma 15/25/50, early stopping)",
        "value": round(ips, 4),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(ips / (1.0 / 45.0), 2),
        "baseline_note": "paper: under 45 s per 512x512 image on an RTX 5000 mobile (context only)",
        "dtype": "f32" if prec == n2f.FP32 else "bf16",
        "data": "synthetic",
        "config": {"workload": f"single {args.size}x{args.size} grayscale, Gaussian sigma 15/25/50 per 255, "
                               "patience 100, one image per step",
                   "precision": args.precision, "global_batch": 1, "image": f"{args.size}x{args.size}x1"},
        "mpx_per_s": round(ips * npx / 1e6, 4),
        "latency_s": {"p50": round(float(np.percentile(lats, 50)), 3), "p99": round(float(np.percentile(lats, 99)), 3)},
        "epochs_mean": round(float(np.mean(epochs)), 1),
        "per_image": psnrs,
        "kernels": kern,
        "roofline": {"bound": "mfma", "kernel": KNAMES[dom], "achieved": round(achieved, 2),
                     "peak": PEAK[args.precision], "unit": "TFLOP/s", "frac": round(achieved / PEAK[args.precision], 4),
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(imgs[1][2], float(np.mean(epochs)))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
