"""Launch-geometry autotuner for grouped batches (BF16).

A grouped launch walks the virtual blocks of every image of a batch with a
fixed number of hardware blocks per kind (n2f_group_grid_set).  The best
number depends on the kind (the 3x3 kernels hold most of a CU's shared
memory, the small kernels are latency-bound) and on the batch's image sizes
(how many virtual blocks there are to balance).  The tuner times each kind
over a few epochs of a representative batch at every candidate grid, keeps
the fastest, and stores the choice per (device, size bucket) in a JSON table
that `apply` loads at start-up.  The geometry never changes results: every
virtual block computes the same values whichever hardware block runs it.

It also picks the weight gradient's split count for batches
(`n2f_config.wgrad_splits`): in a batch the other images already fill the
chip, so fewer, longer splits pay (less per-split overhead, fewer partial
rows for Adam to read).  Unlike the geometry, the split count fixes the order
of the gradient's sums, so runs agree bit for bit only at the same value; the
entry records it and the caller puts it in the batch's configuration.

    python -m paper_2108_10209_amd.autotune --out paper_2108_10209_amd/tuning.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

from . import n2f

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
CANDIDATES = (128, 256, 384, 512, 768, 1024)
SPLIT_CANDIDATES = (0, 32, 16)   # 0: the library default (64 for BF16)


def size_bucket(npix_per_image: float) -> int:
    """log2 of the mean image size in pixels, rounded: images of similar area
    share a tuning entry."""
    return int(round(math.log2(max(npix_per_image, 1.0))))


def _device_name() -> str:
    """Architecture and compute-unit count of device 0 (the marketing name
    is not always available to the runtime)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]} {p.multi_processor_count}CU"


def _time_kinds(batch, epochs: int) -> dict:
    """Per-launch milliseconds of every grouped kind over `epochs` epochs."""
    n2f.profile_begin(1)
    batch.run(max_epochs=epochs)
    out = {}
    for kind in range(len(n2f.GROUP_KINDS)):
        ms, launches, _ = n2f.profile_read(n2f.K_GROUP + kind)
        if launches:
            out[kind] = ms / launches
    n2f.profile_end()
    return out


def tune(images, candidates=CANDIDATES, epochs: int = 2, log=None, split_candidates=SPLIT_CANDIDATES) -> dict:
    """Tune the grid of every grouped kind on `images` (device tensors, C x
    H x W).  The images train for a fixed number of epochs meanwhile, so none
    drops out of the group; the returned entry has the chosen grid and the
    per-launch time before and after for each kind."""
    log = log or (lambda *a: print(*a, file=sys.stderr, flush=True))
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=1000)
    batch = n2f.Batch(images, cfg, n_streams=n2f.BATCH_GROUPED)
    try:
        batch.run(max_epochs=1)                       # first epoch: graph capture, tables
        base = _time_kinds(batch, epochs)
        order = sorted(base, key=lambda k: -base[k])  # largest per-launch time first
        chosen, report = {}, {}
        for kind in order:
            start = n2f.group_grid(kind)
            best_g, best_t = start, base[kind]
            for g in candidates:
                if g == start:
                    continue
                n2f.set_group_grid(kind, g)
                t = _time_kinds(batch, epochs).get(kind)
                if t is not None and t < best_t:
                    best_g, best_t = g, t
            n2f.set_group_grid(kind, best_g)
            chosen[n2f.GROUP_KINDS[kind]] = best_g
            report[n2f.GROUP_KINDS[kind]] = {"grid_before": start, "us_before": round(1e3 * base[kind], 2),
                                             "grid": best_g, "us": round(1e3 * best_t, 2)}
            log(f"  {n2f.GROUP_KINDS[kind]:>18s}: grid {start} -> {best_g}, "
                f"{1e3 * base[kind]:.1f} -> {1e3 * best_t:.1f} us per launch")
    finally:
        batch.close()
    # the weight gradient's split count: whole-epoch kernel time (every kind)
    split_ms = {}
    for k in split_candidates:
        b = n2f.Batch(images, n2f.default_config(precision=n2f.BF16, fixed_epochs=1000, wgrad_splits=k),
                      n_streams=n2f.BATCH_GROUPED)
        try:
            b.run(max_epochs=1)
            n2f.profile_begin(1)
            b.run(max_epochs=epochs)
            split_ms[k] = sum(n2f.profile_read(n2f.K_GROUP + kind)[0] for kind in range(len(n2f.GROUP_KINDS))) / epochs
            n2f.profile_end()
        finally:
            b.close()
        log(f"  wgrad_splits {k}: {split_ms[k]:.2f} ms of kernels per epoch")
    best_split = min(split_ms, key=split_ms.get) if split_ms else 0
    npix = sum(int(x.shape[-2]) * int(x.shape[-1]) for x in images) / len(images)
    return {"device": _device_name(), "precision": "bf16", "bucket": size_bucket(npix),
            "images": len(images), "mean_pixels": round(npix), "group_grid": chosen, "wgrad_splits": best_split,
            "split_ms_per_epoch": {str(k): round(v, 3) for k, v in split_ms.items()}, "report": report}


def load_table(path: str = TABLE) -> list:
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f).get("entries", [])


def save_entry(entry: dict, path: str = TABLE):
    """Insert or replace the entry of the same device, precision and bucket."""
    entries = [e for e in load_table(path)
               if (e["device"], e["precision"], e["bucket"]) != (entry["device"], entry["precision"], entry["bucket"])]
    entries.append(entry)
    entries.sort(key=lambda e: (e["device"], e["precision"], e["bucket"]))
    with open(path, "w") as f:
        json.dump({"entries": entries}, f, indent=1, sort_keys=True)
        f.write("\n")


def apply(npix_per_image: float, path: str = TABLE, device: str | None = None) -> dict | None:
    """Set the grids of the entry for this device whose size bucket is
    nearest to `npix_per_image`; returns that entry (None: no entry, the
    built-in grids stay)."""
    device = device or _device_name()
    entries = [e for e in load_table(path) if e["device"] == device and e["precision"] == "bf16"]
    if not entries:
        return None
    b = size_bucket(npix_per_image)
    e = min(entries, key=lambda e: abs(e["bucket"] - b))
    for name, grid in e["group_grid"].items():
        n2f.set_group_grid(n2f.GROUP_KINDS.index(name), int(grid))
    return e


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--images", type=int, default=64, help="images of the tuning batch")
    ap.add_argument("--min-side", type=int, default=256)
    ap.add_argument("--max-side", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=2, help="epochs timed per candidate")
    args = ap.parse_args(argv)
    import torch
    from . import synth
    pairs = synth.batch_images(args.images, args.min_side, args.max_side, seed=11)
    xs = [torch.from_numpy(x).to("cuda:0") for _, x in pairs]
    print(f"tuning on {len(xs)} images, sides [{args.min_side}, {args.max_side}]", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    entry = tune(xs, epochs=args.epochs)
    entry["tuned_in_s"] = round(time.perf_counter() - t0, 1)
    save_entry(entry, args.out)
    print(json.dumps({k: entry[k] for k in ("device", "bucket", "group_grid", "wgrad_splits", "tuned_in_s")}))


if __name__ == "__main__":
    main()
