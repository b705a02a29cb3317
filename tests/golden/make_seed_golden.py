"""Write the oracle's end-to-end PSNR over several initial-weight seeds.

A single run of the method ends at an epoch that moves with rounding noise
and with the initial weights, so single-run PSNRs of equally correct
implementations differ by a few tenths of a dB; the mean over seeds is the
quantity compared.  Runs the CPU FP64 reference (oracle/n2f_oracle.py) on the
64x64 blobs scene (clean seed 0) with Gaussian noise sigma 25/255 (noise seed
1), early stopping with patience 100, initial weights from SplitMix64 seeds
0..n-1, and stores per-seed PSNR, epochs and best epochs.

    python tests/golden/make_seed_golden.py --seeds 128 --workers 7
    python tests/golden/make_seed_golden.py --seeds 64 --fixed-epochs 8

With --fixed-epochs E the stopping rule is off and the output is the last
validation output after E epochs (the 64x64 configuration of 8 fixed epochs);
the file is then oracle_psnr_64_sigma25_fixedE_seeds.json.

Seeds already stored in the output file are kept and only the missing ones
are run (each worker single-threaded).  Calls only the oracle and the input
generators.
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


FIXED = 0


def run_one(seed):
    from oracle import n2f_oracle as O
    from paper_2108_10209_amd import synth
    clean, noisy = synth.small_64(0)
    t0 = time.time()
    r = O.denoise(noisy, synth.init_params(1, seed), O.Hyper(fixed_epochs=FIXED))
    out = {"seed": seed, "psnr": synth.psnr(r.y, clean), "epochs": r.epochs[0], "best_epoch": r.best_epoch[0],
           "capped": r.capped[0], "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=128)
    ap.add_argument("--workers", type=int, default=7)
    ap.add_argument("--fixed-epochs", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    global FIXED
    FIXED = a.fixed_epochs
    if a.out is None:
        tag = f"_fixed{FIXED}" if FIXED else ""
        a.out = os.path.join(HERE, f"oracle_psnr_64_sigma25{tag}_seeds.json")
    have = {}
    if os.path.exists(a.out):
        have = {r["seed"]: r for r in json.load(open(a.out))["runs"]}
    todo = [s for s in range(a.seeds) if s not in have]
    with Pool(a.workers, initializer=_set_fixed, initargs=(FIXED,)) as pool:
        for r in pool.imap_unordered(run_one, todo):
            have[r["seed"]] = r
            write(a.out, have, FIXED)  # after every seed, so an interrupted run keeps what it finished
    out = write(a.out, have, FIXED)
    print(a.out, len(out["runs"]), out["mean_psnr"], out["std_psnr"])


def _set_fixed(e):
    global FIXED
    FIXED = e


def write(path, have, fixed):
    import numpy as np
    from paper_2108_10209_amd import synth
    runs = [have[s] for s in sorted(have)]
    clean, noisy = synth.small_64(0)
    ps = np.array([r["psnr"] for r in runs])
    mode = f"{fixed} fixed epochs, no stopping rule" if fixed else "early stopping"
    out = {"source": f"CPU FP64 oracle, whole Noise2Fast loop (Methods section), {mode}, "
                     "written by tests/golden/make_seed_golden.py",
           "image": "64x64 blobs, clean seed 0, Gaussian sigma 25/255, noise seed 1", "patience": 100,
           "fixed_epochs": fixed,
           "noisy_psnr": synth.psnr(noisy, clean), "mean_psnr": float(ps.mean()), "std_psnr": float(ps.std(ddof=1)),
           "runs": runs}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
    os.replace(tmp, path)
    return out


if __name__ == "__main__":
    main()
