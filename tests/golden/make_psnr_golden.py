"""Write the oracle's end-to-end result for one synthetic image to JSON.

Runs the CPU FP64 reference (oracle/n2f_oracle.py) through the whole loop of
the paper (train on the four checkerboard pairs, validate every epoch, stop
after 100 epochs without improvement, average the last 100 outputs) on the
blobs scene (clean seed 0) with Gaussian noise sigma/255, initial weights
from SplitMix64 seed 0, and stores PSNR, epochs and the validation history.

    python tests/golden/make_psnr_golden.py --size 512 --sigma 25 --noise-seed 2

Calls only the oracle and the input generators.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import n2f_oracle as O  # noqa: E402
from paper_2108_10209_amd import synth  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--sigma", type=float, default=25)
    ap.add_argument("--noise-seed", type=int, default=2)
    ap.add_argument("--patience", type=int, default=100)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    clean, noisy = synth.single_512(a.sigma, noise_seed=a.noise_seed, size=a.size)
    th0 = synth.init_params(1, 0)
    t0 = time.time()
    epochs_seen = []

    def trace(k, e, p, st, g, loss):
        if p == 3 and (not epochs_seen or epochs_seen[-1] != e):
            epochs_seen.append(e)
            print(f"epoch {e} done, {time.time() - t0:.0f} s", flush=True)

    r = O.denoise(noisy, th0, O.Hyper(patience=a.patience), trace=trace)
    out = {
        "source": "CPU FP64 oracle, whole Noise2Fast loop (Methods section), written by "
                  "tests/golden/make_psnr_golden.py",
        "size": a.size, "sigma255": a.sigma, "clean_seed": 0, "noise_seed": a.noise_seed, "init_seed": 0,
        "patience": a.patience,
        "psnr": synth.psnr(r.y, clean), "noisy_psnr": synth.psnr(noisy, clean),
        "epochs": r.epochs[0], "best_epoch": r.best_epoch[0], "capped": r.capped[0],
        "history": r.history[0], "seconds": time.time() - t0,
    }
    path = a.out or os.path.join(HERE, f"oracle_psnr_{a.size}_sigma{int(a.sigma)}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["psnr"], out["epochs"], out["best_epoch"])


if __name__ == "__main__":
    main()
