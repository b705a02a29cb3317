#!/usr/bin/env python3
"""Throughput of Noise2Fast denoising on one MI355X.

Default workload: a batch of 64 independent grayscale images with sides
uniform in [256, 1024] (blobs scenes, seed 3; Poisson peak 30 + Gaussian
10/255 noise), each trained from scratch with the paper's early-stopping
rule (patience 100) and returned as the mean of the last 100 validation
outputs, BF16 convolutions, grouped launches (one launch per layer covers
every image, one recorded graph per epoch).  One "step" denoises the whole
batch to convergence.  The inputs sit in HBM before the timed region starts.

Prints one JSON line: images/s and Mpx/s, PSNR, the roofline position of
the kernel with the largest summed time (HIP events around every grouped
launch of the sampled epochs), the same images through the plain FP32 path
one at a time, the single 512x512 configuration as a secondary figure, and
the CPU FP64 oracle timed on a bounded sample of the same work.
Other workloads: --workload single | serve | ablation | volume | large.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK = {"fp32": 157.3, "bf16": 2500.0}      # dense MFMA TFLOP/s, MI355X
CONV_FLOP_PER_PX = 2 * 9 * 64 * 64          # one 64->64 3x3 conv pass per pixel
# timed kernel classes: name, algorithmic FLOP per pixel of one launch
KNAMES = {0: "conv3x3_fwd", 1: "conv3x3_backward_layer", 2: "adam"}
KFLOP = {0: CONV_FLOP_PER_PX, 1: 2 * CONV_FLOP_PER_PX, 2: 0}


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


def _psnr_list(outs, cleans):
    from paper_2108_10209_amd import synth
    return [synth.psnr(y.cpu().numpy(), c) for y, c in zip(outs, cleans)]


# grouped launch kinds (n2f.GROUP_KINDS order) whose work is the dense 3x3
# contraction: algorithmic FLOP per pixel of the launch (the fused head and
# first-layer work is small VALU work on top and is not counted)
GROUP_CONV_KINDS = {0: CONV_FLOP_PER_PX, 1: CONV_FLOP_PER_PX, 2: CONV_FLOP_PER_PX, 3: CONV_FLOP_PER_PX,
                    4: CONV_FLOP_PER_PX, 5: CONV_FLOP_PER_PX}
# algorithmic HBM bytes per pixel of the grouped 3x3 kinds (inputs read once, outputs written once):
# forward 128 + 128, data gradient 128 + 8 (ReLU bit mask) + 128, training head 128 + 4 (target) + 128 (delta),
# validation head 128 + 4 + 4, first layer fused into layer 2 4 + 128 + 8 + 128 + 8, weight gradient 128 + 128
GROUP_CONV_BYTES = {0: 256, 1: 264, 2: 260, 3: 136, 4: 276, 5: 256}
HBM_PEAK_GBS = 8000.0
# rocprofv3 symbol prefix of each grouped kind
GROUP_SYMBOL = {0: "k_conv_bf16_group<0>", 1: "k_conv_bf16_group<1>", 2: "k_conv_bf16_group<2>",
                3: "k_conv_bf16_group<3>", 4: "k_conv_bf16_group<4>", 5: "k_wgrad_bf16_group"}


def host_info():
    """Threads the oracle's BLAS uses, and the host CPU model."""
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return int(cores), model, os.cpu_count()


def oracle_sec_per_mpx_epoch(noisy, min_seconds: float = 8.0):
    """The FP64 oracle's seconds per (megapixel x epoch): whole epochs (four
    training steps in table order, then the full-image validation) of one
    image, repeated until at least `min_seconds` of CPU work."""
    from oracle import n2f_oracle as O
    from paper_2108_10209_amd import synth
    h = O.Hyper()
    xs, _, _ = O.standardize(noisy)
    pairs = O.training_pairs(xs)
    st = O.new_state(synth.init_params(1, 0)[0])
    t0 = time.perf_counter()
    epochs = 0
    while True:
        for inp, tgt in pairs:
            st = O.train_step(st, 1, inp, tgt[0], h)[0]
        O.validate(st.theta, 1, xs, 0, h)
        epochs += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    sec = time.perf_counter() - t0
    return sec / (epochs * noisy.shape[1] * noisy.shape[2] / 1e6), sec, epochs


def launch_geometry(args, xs, n2f):
    """Grouped launch geometry for the timed batch (never changes results)."""
    import torch
    from paper_2108_10209_amd import autotune, synth
    src = args.tuning
    entry = None
    if src == "tune":
        t0 = time.perf_counter()
        pairs = synth.batch_images(len(xs), 256, 1024, seed=11)   # other images than the timed ones
        entry = autotune.tune([torch.from_numpy(x).to(xs[0].device) for _, x in pairs])
        print(f"tuned in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    elif src != "none":
        npix = sum(int(x.shape[-2]) * int(x.shape[-1]) for x in xs) / len(xs)
        entry = autotune.apply(npix, autotune.TABLE if src == "auto" else src)
    grids = {name: n2f.group_grid(k) for k, name in enumerate(n2f.GROUP_KINDS)}
    return {"source": src if entry is not None else "built-in", "group_grid": grids,
            "tuning_bucket": entry["bucket"] if entry else None,
            "wgrad_splits": entry.get("wgrad_splits", 0) if entry else 0}


def bench_c3(args):
    """64 independent grayscale images, sides uniform in [256, 1024],
    Poisson (peak 30) + Gaussian (10/255) noise, trained together to their
    own early stops (BF16, grouped launches by default): images/s to
    convergence.  Beside it: the plain FP32 path on the first
    `--fp32-sample` images one at a time, the single 512x512 configuration,
    and the oracle extrapolated per megapixel-epoch."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    dev = torch.device("cuda:0")
    pairs = synth.batch_images(args.batch_n, 256, 1024, seed=3)
    cleans = [c for c, _ in pairs]
    xs = [torch.from_numpy(x).to(dev) for _, x in pairs]
    npx = sum(x.numel() for x in xs)
    prec = n2f.BF16 if args.precision == "bf16" else n2f.FP32
    streams = args.streams if prec == n2f.BF16 else max(args.streams, 1)
    geometry = launch_geometry(args, xs, n2f)
    splits = args.wgrad_splits if args.wgrad_splits >= 0 else (geometry.get("wgrad_splits") or 0)
    if prec != n2f.BF16:
        splits = 0
    geometry["wgrad_splits"] = splits
    cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs, wgrad_splits=splits)
    print(f"batch of {len(xs)} images, {npx / 1e6:.1f} Mpx, streams {streams}, weight-gradient splits "
          f"{splits or 'default'}", file=sys.stderr, flush=True)

    def step():
        b = n2f.Batch(xs, cfg, n_streams=streams)
        b.run()
        outs = [b.result(i) for i in range(len(xs))]
        ep = [b.progress(i)[0] for i in range(len(xs))]
        b.close()
        return outs, ep

    for i in range(args.warmup):
        t0 = time.perf_counter()
        step()
        print(f"warmup {i} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    grouped = streams <= n2f.BATCH_GROUPED
    n2f.profile_begin(args.profile_every)
    t0 = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        outs, epochs = step()
        print(f"step {i} done ({time.perf_counter() - t1:.1f} s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n2f.profile_end()
    ps = _psnr_list(outs, cleans)
    ips = len(xs) * args.steps / wall
    mpx_epochs = sum(x.numel() * e for x, e in zip(xs, epochs)) / 1e6
    # kernel timing: every grouped launch of one epoch in profile_every
    kern, dom = {}, None
    if grouped:
        for kind, name in enumerate(n2f.GROUP_KINDS):
            ms, nl, px = n2f.profile_read(n2f.K_GROUP + kind)
            if nl == 0:
                continue
            kern[name] = {"total_ms_sampled": round(ms, 3), "launches_sampled": nl, "avg_us": round(1e3 * ms / nl, 2)}
            if kind in GROUP_CONV_KINDS:
                kern[name]["tflops"] = round(px * GROUP_CONV_KINDS[kind] / max(ms, 1e-9) / 1e9, 2)
                kern[name]["hbm_gbs"] = round(px * GROUP_CONV_BYTES[kind] / max(ms, 1e-9) / 1e6, 1)
            if dom is None or ms > kern[n2f.GROUP_KINDS[dom]]["total_ms_sampled"]:
                dom = kind
    result = {
        "metric": "images/s denoised to convergence (batch of 64 images, sides U[256,1024], Poisson-Gaussian)",
        "value": round(ips, 4), "unit": "images/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "baseline_note": "the paper has no figure for this workload; its 512x512 timing (under 45 s on an RTX 5000 "
                         "mobile) is context only; the oracle on this host is in cpu_baseline",
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"batch of {len(xs)} independent grayscale images, H and W uniform in [256,1024] "
                               "(blobs scenes, seed 3), Poisson peak 30 + Gaussian 10/255, patience 100, each to its "
                               "own early stop; one step = the whole batch",
                   "precision": args.precision, "launches": ("grouped" if streams == n2f.BATCH_GROUPED else f"grouped on {-streams} streams")
                   if grouped else f"{streams} streams",
                   "images": len(xs), "mpx": round(npx / 1e6, 3)},
        "mpx_per_s": round(npx * args.steps / wall / 1e6, 3),
        "mpx_epochs_per_s": round(mpx_epochs * args.steps / wall, 2),
        "epochs_mean": round(float(np.mean(epochs)), 1),
        "psnr_mean": round(float(np.mean(ps)), 3),
        "noisy_psnr_mean": round(float(np.mean([synth.psnr(x, c) for (c, x) in pairs])), 3),
        "kernels": kern,
        "launch_geometry": geometry,
    }
    if dom is not None:
        k = kern[n2f.GROUP_KINDS[dom]]
        peak = PEAK[args.precision]
        result["roofline"] = {"bound": "mfma", "kernel": GROUP_SYMBOL.get(dom, n2f.GROUP_KINDS[dom]),
                              "achieved": k.get("tflops", 0.0), "peak": peak, "unit": "TFLOP/s",
                              "frac": round(k.get("tflops", 0.0) / peak, 4), "traffic": None}
        if "hbm_gbs" in k:   # the same launches against the HBM roof (algorithmic bytes)
            result["roofline"]["hbm_achieved_gbs"] = k["hbm_gbs"]
            result["roofline"]["hbm_frac"] = round(k["hbm_gbs"] / HBM_PEAK_GBS, 4)
        tr = measured_traffic(GROUP_SYMBOL.get(dom, ""))
        if tr is not None:
            result["roofline"]["traffic"] = tr["bytes_per_launch"]
            result["roofline"]["traffic_detail"] = tr
    # the same images through the plain FP32 path, one at a time
    k32 = min(args.fp32_sample, len(xs))
    if k32 > 0:
        cfg32 = n2f.default_config(precision=n2f.FP32, max_epochs=args.max_epochs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        outs32 = [n2f.denoise(xs[i], cfg32)[0] for i in range(k32)]
        torch.cuda.synchronize()
        wall32 = time.perf_counter() - t1
        ps32 = _psnr_list(outs32, cleans[:k32])
        result["fp32_single_image"] = {
            "images": k32, "images_per_s": round(k32 / wall32, 4),
            "psnr_mean_same_images": round(float(np.mean(ps32)), 3),
            "batched_psnr_mean_same_images": round(float(np.mean(ps[:k32])), 3),
            "batched_speedup_images_per_s": round(ips / (k32 / wall32), 2)}
        print(f"fp32 single-image leg: {k32} images in {wall32:.1f} s", file=sys.stderr, flush=True)
    # the same batch with each image replaying its own epoch graph on 2
    # streams (secondary; timed after the main region, one step, after one
    # warm step): throughput and a check that every image's result is the
    # same bits as in the grouped run
    if args.secondary and grouped:
        def step_streams():
            b = n2f.Batch(xs, cfg, n_streams=2)
            b.run()
            o = [b.result(i) for i in range(len(xs))]
            b.close()
            return o
        step_streams()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        outs2 = step_streams()
        torch.cuda.synchronize()
        wall2 = time.perf_counter() - t1
        result["per_image_graphs_2_streams"] = {
            "images_per_s": round(len(xs) / wall2, 4),
            "mpx_epochs_per_s": round(mpx_epochs / wall2, 2),
            "same_bits_as_grouped": all(torch.equal(a, b) for a, b in zip(outs, outs2)),
            "note": "each image replays its own epoch graph, two streams; launches of different kinds overlap "
                    "across the streams, which the grouped launches (one kind at a time) do not; per-kernel "
                    "rates are not separable there, so the roofline above is taken from the grouped run"}
        print(f"2-stream leg: {wall2:.1f} s", file=sys.stderr, flush=True)
    # the single 512x512 configuration (secondary)
    if args.secondary:
        imgs = []
        for i, sg in enumerate([15, 25, 50]):
            clean, noisy = synth.single_512(sg, noise_seed=i + 1, size=512)
            imgs.append((sg, clean, noisy, torch.from_numpy(noisy).to(dev)))
        a2 = argparse.Namespace(**vars(args))
        a2.steps, a2.warmup, a2.size = 3, 1, 512
        single = {}
        for pname in ("bf16", "fp32"):
            r = run_single(a2, imgs, pname, profile=False)
            single[pname] = {"images_per_s": round(r["ips"], 4), "epochs_mean": r["epochs_mean"],
                             "psnr": [p["psnr"] for p in r["per_image"]],
                             "ms_per_epoch": round(1e3 * r["wall"] / max(1, sum(p["epochs"] for p in r["per_image"])), 4)}
        result["single_512"] = {"workload": "512x512 grayscale blobs, Gaussian sigma 15/25/50, one image at a time",
                                **single}
        print("single 512 done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        med = int(np.argsort([x.numel() for x in xs])[len(xs) // 2])
        spe, sec, ne = oracle_sec_per_mpx_epoch(pairs[med][1])
        cores, model, ncpu = host_info()
        batch_sec = spe * mpx_epochs
        result["cpu_baseline"] = {
            "value": round(len(xs) / batch_sec, 6), "unit": "images/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_cpus": ncpu, "sec_per_mpx_epoch": round(spe, 3),
            "sample": f"{ne} whole epoch(s) (4 training steps + validation) of batch image {med} "
                      f"({pairs[med][1].shape[1]}x{pairs[med][1].shape[2]}, the median size) in {sec:.1f} s, "
                      f"extrapolated per megapixel-epoch to the batch's {mpx_epochs:.0f} Mpx-epochs "
                      "(the GPU run's epochs to convergence)"}
        result["speedup_vs_cpu_oracle"] = round(ips / result["cpu_baseline"]["value"], 1)
    return result


# Table 1 of the paper (BSD68, PSNR dB): normal, 2x2 blocks ("Quad"), exact
# targets ("Exact"); context for the synthetic comparison below
PAPER_TABLE1 = {"sigma25": {"normal": 28.12, "quad": 27.56, "exact": 28.12},
                "sigma50": {"normal": 25.23, "quad": 24.97, "exact": 25.24}}


def bench_ablation(args):
    """The ablation study (Methods, Ablation Study; Table 1) on synthetic
    512x512 scenes: the checkerboard method, 2x2-block downsampling, and
    exact targets (known signal difference removed), each trained to its
    own early stop on the same noisy images.  Reports PSNR per variant and
    its difference from the checkerboard run, and images/s per variant."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    dev = torch.device("cuda:0")
    prec = n2f.BF16 if args.precision == "bf16" else n2f.FP32
    variants = {"normal": dict(), "quad": dict(downsample=n2f.DS_QUAD), "exact": dict(exact_targets=1)}
    S = args.size
    scenes = {"blobs": synth.blobs(S, S, 0), "microscopy": synth.microscopy(S, S, 4)}
    seeds = list(range(1, args.ablation_seeds + 1))
    rows, wall = {}, {v: 0.0 for v in variants}
    nimg = {v: 0 for v in variants}
    for scene, clean in scenes.items():
        for sg in (25, 50):
            cell = {}
            for name, kw in variants.items():
                cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs, **kw)
                ps, eps = [], []
                for sd in seeds:
                    noisy = synth.add_gaussian(clean, sg / 255.0, 1000 * sg + sd)
                    x = torch.from_numpy(noisy).to(dev)
                    c = torch.from_numpy(np.ascontiguousarray(clean, np.float32)).to(dev)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    run = n2f.Run(x, cfg)
                    if kw.get("exact_targets"):
                        run.set_clean(c)
                    run.run_epochs(0, args.max_epochs)
                    y = run.result()
                    torch.cuda.synchronize()
                    wall[name] += time.perf_counter() - t0
                    nimg[name] += 1
                    eps.append(run.progress(0)[0])
                    run.close()
                    ps.append(synth.psnr(y.cpu().numpy(), clean))
                cell[name] = {"psnr": round(float(np.mean(ps)), 3),
                              "psnr_sd": round(float(np.std(ps, ddof=1)), 3) if len(ps) > 1 else None,
                              "epochs_mean": round(float(np.mean(eps)), 1)}
                print(f"{scene} sigma {sg} {name}: {cell[name]}", file=sys.stderr, flush=True)
            for name in ("quad", "exact"):
                cell[name]["delta_db"] = round(cell[name]["psnr"] - cell["normal"]["psnr"], 3)
            cell["noisy_psnr"] = round(float(np.mean([synth.psnr(synth.add_gaussian(clean, sg / 255.0, 1000 * sg + sd),
                                                                  clean) for sd in seeds])), 3)
            rows[f"{scene}_sigma{sg}"] = cell
    ips = {v: round(nimg[v] / wall[v], 4) for v in variants}
    total = sum(nimg.values()) / sum(wall.values())
    return {
        "metric": "images/s denoised to convergence, ablation variants (512x512, sigma 25/50, early stopping)",
        "value": round(total, 4), "unit": "images/s", "n_gpus": 1, "steps": sum(nimg.values()), "warmup": 0,
        "ms_per_step": round(1e3 * sum(wall.values()) / sum(nimg.values()), 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"ablation: checkerboard vs 2x2 blocks vs exact targets, {S}x{S} blobs and "
                               f"microscopy scenes, Gaussian sigma 25 and 50, {len(seeds)} noise seeds each",
                   "precision": args.precision},
        "images_per_s": ips, "psnr": rows, "paper_table1_bsd68_context": PAPER_TABLE1,
    }


# the paper's live-cell time-lapse (Methods, Fluorescence Microscopy Images):
# 1024x1024 slices, 20 um deep at 0.5 um (41 planes), every 5 min for 24 h
VIDEO_TIMEPOINTS = 24 * 60 // 5 + 1
PAPER_VIDEO_DAYS_V100 = 0.7


def bench_volume(args):
    """One time point of the live-cell time-lapse: a two-channel z-stack
    (nuclear and actin channels, `--volume-z` planes of `--volume-size`^2,
    Poisson peak 10 + Gaussian 0.02 noise) is denoised slice by slice as
    one batch, then each channel is max projected.  Reports slices/s, the
    time per time point, that time scaled to the whole 289-point video,
    and the PSNR of the projections against the clean projections."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    dev = torch.device("cuda:0")
    Z, S = args.volume_z, args.volume_size
    clean = synth.cell_volume(Z, S, S, seed=6)
    noisy = np.stack([synth.add_poisson_gaussian(clean[c], 10.0, 0.02, 60 + c) for c in range(2)])
    xs = [torch.from_numpy(np.ascontiguousarray(noisy[c, z][None])).to(dev) for c in range(2) for z in range(Z)]
    prec = n2f.BF16 if args.precision == "bf16" else n2f.FP32
    cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs)
    print(f"volume: 2 channels x {Z} planes of {S}x{S}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = n2f.Batch(xs, cfg, n_streams=args.streams)
    active = len(xs)
    while active:
        active = b.run(25)
        print(f"  {active} slices still training after {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    den = torch.empty((2, Z, S, S), dtype=torch.float32, device=dev)
    for i in range(len(xs)):
        den[i // Z, i % Z].copy_(b.result(i)[0])
    proj = torch.stack([n2f.max_project(den[c]) for c in range(2)])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    epochs = [b.progress(i)[0] for i in range(len(xs))]
    b.close()
    cp = clean.max(axis=1)
    pn = noisy.max(axis=1)
    pr = proj.cpu().numpy()
    per_tp = wall
    return {
        "metric": "z-slices/s denoised to convergence and max projected (live-cell volume, 2 channels)",
        "value": round(len(xs) / wall, 4), "unit": "slices/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * wall, 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"one time point: 2 channels x {Z} planes of {S}x{S} (synthetic nuclei and actin), "
                               "Poisson peak 10 + Gaussian 0.02, slices as one batch, then max projection",
                   "precision": args.precision, "streams": args.streams},
        "epochs_mean": round(float(np.mean(epochs)), 1),
        "seconds_per_timepoint": round(per_tp, 2),
        "video_hours_extrapolated": round(per_tp * VIDEO_TIMEPOINTS / 3600.0, 2) if (Z, S) == (41, 1024) else None,
        "paper_video_days_v100_context": PAPER_VIDEO_DAYS_V100,
        "projection_psnr": {c: round(synth.psnr(pr[i], cp[i]), 3) for i, c in enumerate(["nuclear", "actin"])},
        "noisy_projection_psnr": {c: round(synth.psnr(pn[i], cp[i]), 3) for i, c in enumerate(["nuclear", "actin"])},
    }


def bench_large(args):
    """One large microscopy-like image (2048x2048: 2000 PSF spots and 30
    filaments, 16-bit levels; Poisson peak 10 + Gaussian 0.02), denoised to
    convergence with BF16 and with FP32 convolutions from `--large-seeds`
    initial weight draws each: images/s, epochs and PSNR (mean and sd over
    the draws, since one run's PSNR moves with its stopping epoch)."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    S = args.large_size
    clean = synth.microscopy(S, S, 4)
    noisy = synth.add_poisson_gaussian(clean, 10.0, 0.02, 40)
    if args.large_crop:   # the centre crop: same scene statistics (sparsity) at a smaller size
        c0 = (S - args.large_crop) // 2
        clean = np.ascontiguousarray(clean[:, c0:c0 + args.large_crop, c0:c0 + args.large_crop])
        noisy = np.ascontiguousarray(noisy[:, c0:c0 + args.large_crop, c0:c0 + args.large_crop])
    x = torch.from_numpy(noisy).to("cuda:0")
    out = {}
    for prec_name, prec in (("bf16", n2f.BF16), ("fp32", n2f.FP32)):
        runs = []
        for seed in range(args.large_seeds):
            cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs, init_seed=seed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run = n2f.Run(x, cfg)
            done = False
            while not done:
                done, _ = run.run_epochs(0, 20)
                print(f"{prec_name} seed {seed}: {run.progress(0)[0]} epochs after {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            y = run.result()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            e, be, _, _ = run.progress(0)
            runs.append({"seconds": round(wall, 2), "epochs": e, "best_epoch": be,
                         "psnr": round(synth.psnr(y.cpu().numpy(), clean), 3)})
            run.close()
        ps = [r["psnr"] for r in runs]
        out[prec_name] = {"images_per_s": round(len(runs) / sum(r["seconds"] for r in runs), 4),
                          "ms_per_epoch": round(1e3 * sum(r["seconds"] for r in runs) / sum(r["epochs"] for r in runs), 2),
                          "psnr_mean": round(float(np.mean(ps)), 3),
                          "psnr_sd": round(float(np.std(ps, ddof=1)), 3) if len(ps) > 1 else None, "runs": runs}
    return {
        "metric": "images/s denoised to convergence (2048x2048 microscopy-like, Poisson-Gaussian)",
        "value": out["bf16"]["images_per_s"], "unit": "images/s", "n_gpus": 1, "steps": args.large_seeds,
        "warmup": 0, "ms_per_step": round(1e3 / out["bf16"]["images_per_s"], 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": (f"centre {args.large_crop}x{args.large_crop} crop of " if args.large_crop else "") +
                               f"one {S}x{S} microscopy-like image (2000 spots, 30 filaments, 16-bit), Poisson peak 10 "
                               f"+ Gaussian 0.02, patience 100; BF16 and FP32 convolutions, {args.large_seeds} "
                               "initial weight draws each",
                   "precision": "bf16 and fp32"},
        "noisy_psnr": round(synth.psnr(noisy, clean), 3), "bf16": out["bf16"], "fp32": out["fp32"],
        "psnr_bf16_minus_fp32": round(out["bf16"]["psnr_mean"] - out["fp32"]["psnr_mean"], 3),
        "speedup_bf16_vs_fp32": round(out["bf16"]["images_per_s"] / out["fp32"]["images_per_s"], 2),
    }


def bench_serve(args):
    """Poisson-arrival stream of `--serve-n` requests (the seeded trace:
    sides log-uniform in [128, 2048], 30% RGB, Gaussian or Poisson noise per
    request) served in real time by the continuous-batching server (BF16,
    grouped launches by default); p50/p99 latency = completion - arrival.
    `--rate 0` calibrates the arrival rate first: the first `--calib-n`
    requests are served as one closed burst and the rate is set to 0.8 x the
    measured capacity (recorded in the output).  Baseline: the plain FP32
    path serving the same trace one request at a time in arrival order,
    simulated from the measured FP32 service times of a stratified sample of
    `--serve-fp32-n` requests (evenly spaced in work = pixels x channels;
    each other request takes the service time of the sampled one nearest in
    work, scaled by the work ratio)."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    dev = torch.device("cuda:0")
    prec = n2f.BF16 if args.precision == "bf16" else n2f.FP32
    grouped = prec == n2f.BF16 and args.streams < 0
    streams = args.streams if args.streams > 0 else 2
    cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs)
    base = synth.serving_trace(n=args.serve_n, rate=1.0, seed=5)
    print(f"generating {len(base)} request images", file=sys.stderr, flush=True)
    data = [synth.request_image(r) for r in base]
    xs = [torch.from_numpy(x).to(dev) for _, x in data]
    work = np.array([r.H * r.W * r.C for r in base], np.float64)

    def serve(ids, arrivals):
        """Serve requests `ids` arriving at `arrivals` (s after start, sorted);
        returns completion times and outputs."""
        srv = n2f.Server(args.arena_gib << 30, cfg, n_streams=streams, max_active=args.max_active, grouped=grouped)
        outs = {i: torch.empty_like(xs[i]) for i in ids}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nxt, done, last = 0, {}, t0
        while len(done) < len(ids):
            now = time.perf_counter() - t0
            while nxt < len(ids) and arrivals[nxt] <= now:
                srv.submit(ids[nxt], xs[ids[nxt]], outs[ids[nxt]])
                nxt += 1
            active, queued = srv.step(args.epochs_per_step) if (nxt > len(done)) else (0, 0)
            if active == 0 and queued == 0 and nxt < len(ids):
                time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
            for rid, st in srv.poll():
                done[rid] = time.perf_counter() - t0
            if time.perf_counter() - last > 30:
                last = time.perf_counter()
                print(f"  {len(done)}/{len(ids)} done, {active} active, {queued} queued at {now:.0f} s",
                      file=sys.stderr, flush=True)
        srv.close()
        return done, outs

    if args.serve_phase == "baseline":
        # FP32 service times of the stratified sample only (written to
        # --fp32-times for a later run of the trace), and the calibration
        pass
    rate, calib = args.rate, None
    if rate <= 0:
        ids = list(range(min(args.calib_n, len(base))))
        done, _ = serve(ids, [0.0] * len(ids))
        cap = len(ids) / max(done.values())
        rate = 0.8 * cap
        calib = {"requests": len(ids), "seconds": round(max(done.values()), 2), "capacity_req_per_s": round(cap, 4)}
        print(f"calibration: capacity {cap:.3f} req/s -> rate {rate:.3f}/s", file=sys.stderr, flush=True)
    arrivals = [r.arrival / rate for r in base]     # the trace's unit-rate arrivals, scaled
    if args.serve_phase == "baseline":
        done, outs = {}, {}
        lat, span, ps = np.zeros(1), 1.0, [float("nan")] * len(base)
    else:
        print(f"serving {len(base)} requests at {rate:.3f}/s", file=sys.stderr, flush=True)
        done, outs = serve(list(range(len(base))), arrivals)
        lat = np.array([done[i] - arrivals[i] for i in range(len(base))])
        span = max(done.values()) - arrivals[0]
        ps = [synth.psnr(outs[i].cpu().numpy(), data[i][0]) for i in range(len(base))]
    result = {
        "metric": "served images/s and p50/p99 request latency (Poisson arrivals, sides log-uniform [128,2048], 30% RGB)",
        "value": round(len(base) / span, 4), "unit": "images/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * span, 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"first {len(base)} requests of the seeded trace (seed 5), Poisson arrivals at "
                               f"{rate:.4f}/s", "precision": args.precision,
                   "launches": f"grouped, {streams} streams" if grouped else f"{streams} streams",
                   "max_active": args.max_active,
                   "epochs_per_step": args.epochs_per_step},
        "rate_req_per_s": round(rate, 4), "calibration": calib,
        "latency_s": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3)},
        "psnr_mean": round(float(np.mean(ps)), 3),
    }
    k = min(args.serve_fp32_n, len(base))
    svc, ps32 = {}, {}
    if args.fp32_times and os.path.exists(args.fp32_times) and args.serve_phase != "baseline":
        saved = json.load(open(args.fp32_times))
        svc = {int(i): v for i, v in saved["seconds"].items()}
        ps32 = {int(i): v for i, v in saved["psnr"].items()}
        k = len(svc)
    elif k > 0:
        order = np.argsort(work)
        sample = sorted(set(int(order[int(round(q))]) for q in np.linspace(0, len(base) - 1, k)))
        cfg32 = n2f.default_config(precision=n2f.FP32, max_epochs=args.max_epochs)
        for j, i in enumerate(sample):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            y32 = n2f.denoise(xs[i], cfg32)[0]
            torch.cuda.synchronize()
            svc[i] = time.perf_counter() - t1
            ps32[i] = synth.psnr(y32.cpu().numpy(), data[i][0])
            if j % 8 == 7:
                print(f"  fp32 sample {j + 1}/{len(sample)}", file=sys.stderr, flush=True)
        if args.fp32_times:
            with open(args.fp32_times, "w") as f:
                json.dump({"seconds": svc, "psnr": ps32, "trace_requests": len(base)}, f)
    if args.serve_phase == "baseline":
        result["phase"] = "baseline (calibration and FP32 sample only; value and latency are not measured here)"
        result["fp32_sample_seconds"] = {str(i): round(v, 3) for i, v in svc.items()}
        return result
    if svc:
        sample = sorted(svc)
        sw = np.array([work[i] for i in sample])
        st = np.array([svc[i] for i in sample])

        def service(i):   # nearest sampled request in work, scaled by the work ratio
            j = int(np.argmin(np.abs(np.log(sw) - np.log(work[i]))))
            return st[j] * work[i] / sw[j]
        comp, t = [], 0.0
        for i in range(len(base)):
            t = max(t, arrivals[i]) + (svc[i] if i in svc else service(i))
            comp.append(t)
        lat32 = np.array([comp[i] - arrivals[i] for i in range(len(base))])
        result["fp32_sequential"] = {
            "sampled_requests": len(sample), "images_per_s": round(len(base) / (comp[-1] - arrivals[0]), 4),
            "latency_s": {"p50": round(float(np.percentile(lat32, 50)), 3),
                          "p99": round(float(np.percentile(lat32, 99)), 3)},
            "psnr_mean_sampled": round(float(np.mean([ps32[i] for i in sample])), 3),
            "served_psnr_mean_sampled": round(float(np.mean([ps[i] for i in sample])), 3),
            "method": "FCFS in arrival order; service times measured on the stratified sample, the others taken "
                      "from the nearest sampled request in work scaled by the work ratio"}
    return result


def bench_single(args):
    """512x512 grayscale images (blobs scene, seed 0) with Gaussian noise
    sigma 15, 25 and 50 (/255, noise seeds 1, 2, 3), each trained from
    scratch to its early stop; one step denoises one image; steps cycle
    through the noise levels.  Roofline of the forward 3x3 convolution
    (timed over runs of consecutive launches)."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth

    dev = torch.device("cuda:0")
    sigmas = [15, 25, 50]
    imgs = []
    for i, sg in enumerate(sigmas):
        clean, noisy = synth.single_512(sg, noise_seed=i + 1, size=args.size)
        imgs.append((sg, clean, noisy, torch.from_numpy(noisy).to(dev)))
    head = args.precision
    runs = {head: run_single(args, imgs, head, profile=True)}
    if not args.no_fp32 and head != "fp32":
        runs["fp32"] = run_single(args, imgs, "fp32", profile=False)
    r = runs[head]
    prof = r["prof"]
    # the forward 3x3 convolution has the largest summed kernel time of any
    # single kernel (rocprofv3 kernel trace); the backward class is a pair
    dom = 0
    ms, nl, px = prof[dom]
    achieved = px * CONV_FLOP_PER_PX / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    kern = {}
    for c in KNAMES:
        ms_c, n_c, px_c = prof[c]
        kern[KNAMES[c]] = {"total_ms_sampled": round(ms_c, 3), "launches_sampled": n_c,
                           "avg_us": round(1e3 * ms_c / max(n_c, 1), 2)}
        if KFLOP[c]:
            kern[KNAMES[c]]["tflops"] = round(px_c * KFLOP[c] / max(ms_c, 1e-9) / 1e9, 2)
    npx = args.size * args.size
    result = {
        "metric": "images/s denoised to convergence (512x512 grayscale, sigma 15/25/50, early stopping)",
        "value": round(r["ips"], 4),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["wall"] / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "baseline_note": "paper: under 45 s per 512x512 image on an RTX 5000 mobile (other hardware and data: "
                         "context only)",
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"single {args.size}x{args.size} grayscale, Gaussian sigma 15/25/50 per 255, "
                               "patience 100, one image per step",
                   "precision": head, "global_batch": 1, "image": f"{args.size}x{args.size}x1"},
        "mpx_per_s": round(r["ips"] * npx / 1e6, 4),
        # per-epoch time: the kernel-speed figure (images/s also moves with
        # the stopping epoch, which any change of rounding shifts)
        "ms_per_epoch": round(1e3 * r["wall"] / max(1, sum(p["epochs"] for p in r["per_image"])), 4),
        "latency_s": r["latency"],
        "epochs_mean": r["epochs_mean"],
        "per_image": r["per_image"],
        "kernels": kern,
        "roofline": {"bound": "mfma", "kernel": KNAMES[dom], "achieved": round(achieved, 2),
                     "peak": PEAK[head], "unit": "TFLOP/s", "frac": round(achieved / PEAK[head], 4),
                     "traffic": None},
    }
    tr = measured_traffic(KERNEL_SYMBOL[head])
    if tr is not None:
        result["roofline"]["traffic"] = tr["bytes_per_launch"]
        result["roofline"]["traffic_detail"] = tr
    for k, v in runs.items():
        if k != head:
            result[k] = {"value": round(v["ips"], 4), "unit": "images/s", "epochs_mean": v["epochs_mean"],
                         "per_image": v["per_image"], "ms_per_step": round(1e3 * v["wall"] / args.steps, 2)}
    if not args.no_cpu_baseline:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(imgs[1][2], float(r["epochs_mean"]))
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="bf16")
    ap.add_argument("--no-fp32", action="store_true", help="single: skip the FP32 comparison run")
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--max-epochs", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", dest="secondary", action="store_false",
                    help="batch: skip the single 512x512 secondary figure")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time the kernels of one epoch in N with HIP events")
    ap.add_argument("--workload", choices=["batch", "single", "serve", "ablation", "volume", "large"],
                    default="batch")
    ap.add_argument("--ablation-seeds", type=int, default=3)
    ap.add_argument("--volume-z", type=int, default=41)
    ap.add_argument("--volume-size", type=int, default=1024)
    ap.add_argument("--large-size", type=int, default=2048)
    ap.add_argument("--large-seeds", type=int, default=3)
    ap.add_argument("--large-crop", type=int, default=0, help="large: denoise the centre crop of this side instead")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--wgrad-splits", type=int, default=-1,
                    help="batch: most pixel splits of a 64->64 weight gradient (0: the library default; -1: the "
                         "tuning table's choice)")
    ap.add_argument("--tuning", default="auto",
                    help="batch: grouped launch geometry: 'auto' (the package's tuning table, when it has an entry "
                         "for this device), 'none' (built-in grids), 'tune' (tune on other images first), or a path")
    ap.add_argument("--streams", type=int, default=-1,
                    help="batch: -1 grouped launches on the caller's stream, -K grouped on K streams (K = 2..4), "
                         ">= 1 per-image graphs on that many streams, 0 in turn")
    ap.add_argument("--fp32-sample", type=int, default=8)
    ap.add_argument("--serve-n", type=int, default=500)
    ap.add_argument("--serve-fp32-n", type=int, default=48)
    ap.add_argument("--calib-n", type=int, default=32)
    ap.add_argument("--serve-phase", choices=["all", "baseline"], default="all",
                    help="serve: 'baseline' only calibrates the rate and times the FP32 sample")
    ap.add_argument("--fp32-times", default="", help="serve: JSON of FP32 sample service times (written by the "
                                                    "baseline phase, read by a later full run)")
    ap.add_argument("--rate", type=float, default=0.0, help="serve: arrivals per s (0: calibrate to 0.8 x capacity)")
    ap.add_argument("--arena-gib", type=int, default=128)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--epochs-per-step", type=int, default=2)
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
    res = {"batch": bench_c3, "single": bench_single, "serve": bench_serve, "ablation": bench_ablation,
           "volume": bench_volume, "large": bench_large}[args.workload](args)
    print(json.dumps(res), flush=True)


def run_single(args, imgs, precision, profile):
    """Time args.steps whole-image denoises (after args.warmup untimed ones)."""
    import numpy as np
    import torch
    from paper_2108_10209_amd import n2f, synth
    prec = n2f.BF16 if precision == "bf16" else n2f.FP32
    cfg = n2f.default_config(precision=prec, max_epochs=args.max_epochs)
    ws = torch.empty(n2f.workspace_bytes(args.size, args.size, 1, cfg), dtype=torch.uint8, device="cuda:0")

    def step(i):
        sg, clean, noisy, x = imgs[i % len(imgs)]
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
        print(f"{precision} warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if profile:
        n2f.profile_begin(args.profile_every)
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step(i))
        print(f"{precision} step {i} done: {outs[-1][1]} epochs, {outs[-1][3]:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = None
    if profile:
        n2f.profile_end()
        prof = {c: n2f.profile_read(c) for c in KNAMES}
    per, epochs, lats = [], [], []
    for i, (y, e, be, lat, status) in enumerate(outs):
        sg, clean, noisy, _ = imgs[i % len(imgs)]
        per.append({"sigma": sg, "psnr": round(synth.psnr(y.cpu().numpy(), clean), 3),
                    "noisy_psnr": round(synth.psnr(noisy, clean), 3), "epochs": e, "best_epoch": be,
                    "capped": status == n2f.WCAPPED})
        epochs.append(e)
        lats.append(lat)
    return {"ips": args.steps / wall, "wall": wall, "prof": prof, "per_image": per,
            "epochs_mean": round(float(np.mean(epochs)), 1),
            "latency": {"p50": round(float(np.percentile(lats, 50)), 3),
                        "p99": round(float(np.percentile(lats, 99)), 3)}}


# kernel symbol prefix of each (precision, class), as rocprofv3 names them
KERNEL_SYMBOL = {"bf16": "k_conv_bf16<0>", "fp32": "k_conv_f32<0>"}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic.md")
CONV_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2108_10209_amd", "csrc", "n2f_conv.hip")


def measured_traffic(symbol):
    """HBM bytes per launch of `symbol` from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on other kernel source."""
    import hashlib
    try:
        src = hashlib.sha256(open(CONV_SRC, "rb").read()).hexdigest()[:16]
        for line in open(TRAFFIC_FILE):
            if line.startswith("traffic:"):
                kv = dict(tok.split("=", 1) for tok in line.split()[1:])
                if kv.get("kernel") == symbol and kv.get("src_sha256_16") == src:
                    return {"fetch_bytes_per_launch": float(kv["fetch_bytes"]),
                            "write_bytes_per_launch": float(kv["write_bytes"]),
                            "bytes_per_launch": float(kv["fetch_bytes"]) + float(kv["write_bytes"]),
                            "algorithmic_bytes_per_launch": float(kv["algorithmic_bytes"])}
    except (OSError, ValueError, KeyError):
        pass
    return None


if __name__ == "__main__":
    main()
