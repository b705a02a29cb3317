"""The large microscopy-like image at its full size (2048x2048, Poisson
peak 10 + Gaussian 0.02), in the launch configuration the benchmark uses.
The oracle cannot run the whole image in a test, so it is checked where it
can be computed exactly: the downsamples bit-exact over the whole image,
and the validation forward on sampled crops. An output pixel depends only on
the 17x17 input window around it (eight 3x3 layers), so the oracle's output
on a crop padded by 8 pixels (image borders keep their zero padding) equals
the full image's output on the crop's core."""
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
S = 2048
R = 8                     # receptive-field radius of the eight 3x3 layers


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def image():
    clean = synth.microscopy(S, S, 4)
    return clean, synth.add_poisson_gaussian(clean, 10.0, 0.02, 40)


def test_large_downsample_bit_exact(image):
    say("2048 downsample")
    _, noisy = image
    r = n2f.Run(torch.from_numpy(noisy).to(DEV))
    xs = r.image(4).cpu().numpy()
    ue, uo = O.checkerboard_up(xs.astype(np.float64))
    le, lo = O.checkerboard_left(xs.astype(np.float64))
    for which, ref in enumerate([ue, uo, le, lo]):
        np.testing.assert_array_equal(r.image(which).cpu().numpy(), ref.astype(np.float32))


# crops: top-left corner, bottom-right corner, a top edge, a left edge, interior
CROPS = [(0, 0), (S - 24, S - 24), (0, 1000), (777, 0), (1031, 1517)]


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_large_validation_forward_on_sampled_crops(image, prec):
    say("2048 validation crops", prec)
    _, noisy = image
    r = n2f.Run(torch.from_numpy(noisy).to(DEV), n2f.default_config(precision=prec))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    r.validate(0)
    y = r.image(5).cpu().numpy()
    th = synth.init_params(1, 0)[0]
    tol = 1e-5 if prec == n2f.FP32 else 2e-2
    for (y0, x0) in CROPS:
        y1, x1 = min(S, y0 + 24), min(S, x0 + 24)
        a0, b0, a1, b1 = max(0, y0 - R), max(0, x0 - R), min(S, y1 + R), min(S, x1 + R)
        y_or, _ = O.validate(th, 1, xs[:, a0:a1, b0:b1], 0, O.Hyper())
        core = y_or[y0 - a0:y1 - a0, x0 - b0:x1 - b0]
        err = rel(y[y0:y1, x0:x1], core)
        say("  crop", y0, x0, "rel", err)
        assert err < tol, (y0, x0, err)
