"""Degenerate image sizes on the GPU against the CPU FP64 oracle, through
the C ABI: the smallest images the method accepts (2x2, whose checkerboard
images are 2x1 and 1x2 and whose 2x2-block images are single pixels), odd
sizes of 3, and strips two pixels tall or three wide, each with one and
three channels.  FP32 after two fixed epochs within 1e-4 of the oracle;
BF16 the first step within 2e-2 per tensor, of the exact gradient or, for a
tensor that BF16 rounding alone moves by more than 1e-2, of a model of the
path's rounding (see `bf16_bar`), and a finite output.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth
from bf16_bar import bf16_check, summary

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H0 = O.Hyper()
SHAPES = [(1, 2, 2), (3, 2, 2), (1, 2, 3), (1, 3, 2), (1, 3, 3), (3, 3, 3), (1, 2, 100), (1, 100, 3), (2, 5, 2)]


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def tiny_image(C, H, W):
    rng = np.random.default_rng(100 * C + 10 * H + W)
    return rng.uniform(0.0, 1.0, (C, H, W)).astype(np.float32)


@pytest.mark.parametrize("ds", ["checkerboard", "quad"])
@pytest.mark.parametrize("C,H,W", SHAPES)
def test_tiny_fp32_fixed_epochs_match_oracle(C, H, W, ds):
    say("tiny fp32", ds, C, H, W)
    x = tiny_image(C, H, W)
    mode = n2f.DS_QUAD if ds == "quad" else n2f.DS_CHECKERBOARD
    y, st = n2f.denoise(dev(x), n2f.default_config(fixed_epochs=2, downsample=mode))
    assert st == n2f.OK
    ref = O.denoise(x, synth.init_params(C, 0), O.Hyper(fixed_epochs=2), downsample=ds)
    for k in range(C):
        assert rel(y[k].cpu().numpy(), ref.y[k]) < 1e-4, k


@pytest.mark.parametrize("ds", ["checkerboard", "quad"])
@pytest.mark.parametrize("C,H,W", SHAPES)
def test_tiny_bf16_first_step_and_finite_output(C, H, W, ds):
    say("tiny bf16", ds, C, H, W)
    x = tiny_image(C, H, W)
    mode = n2f.DS_QUAD if ds == "quad" else n2f.DS_CHECKERBOARD
    cfg = n2f.default_config(fixed_epochs=2, downsample=mode, precision=n2f.BF16)
    r = n2f.Run(dev(x), cfg)
    xs = r.image(4).cpu().numpy().astype(np.float64)
    pairs = O.training_pairs(xs, ds)
    th0 = synth.init_params(C, 0)
    for k in range(C):
        r.train_step(k, 0)
        g, loss = r.get_grad(k)
        th = th0[k].astype(np.float64)
        _, g_or, loss_or, _ = O.train_step(O.new_state(th), C, pairs[0][0], pairs[0][1][k], H0)
        # a few pixels of pure noise make near-cancelling gradient sums:
        # ill-conditioned tensors are judged against the BF16 rounding model
        ok, rows = bf16_check(g, th, C, pairs[0][0], pairs[0][1][k])
        say("  " + summary(rows))
        assert ok, rows
        assert abs(loss - loss_or) / abs(loss_or) < 2e-2
    y, st = n2f.denoise(dev(x), cfg)
    assert st == n2f.OK and torch.isfinite(y).all()
