"""Many independent images on one GPU: a batch of uneven sizes and the
continuous-batching server.  Each image's result must be the same bits as
the image denoised alone (every run's kernels are deterministic and touch
only that run's workspace, whatever else is on the device)."""
import sys

import numpy as np
import pytest
import torch

from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)


SHAPES = [(1, 96, 80), (1, 64, 130), (1, 121, 72), (1, 50, 66), (3, 40, 44), (1, 33, 35)]


def _images(shapes, seed=0):
    out = []
    for i, (C, H, W) in enumerate(shapes):
        clean = synth.blobs(H, W, seed + i, C=C)
        out.append(synth.add_gaussian(clean, 25 / 255, seed + 50 + i))
    return out


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
@pytest.mark.parametrize("kw", [dict(fixed_epochs=5), dict(patience=5, max_epochs=60)])
def test_batch_equals_alone(prec, kw):
    say("batch", prec, kw)
    imgs = _images(SHAPES)
    cfg = n2f.default_config(precision=prec, **kw)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=3)
    assert b.run() == 0
    for i, x in enumerate(imgs):
        yb = b.result(i)
        ya, st = n2f.denoise(dev(x), cfg)
        assert torch.equal(yb, ya), i
        assert b.progress(i)[1]


def test_batch_constant_image_and_max_epochs():
    imgs = _images(SHAPES[:3])
    imgs[1] = np.full_like(imgs[1], 0.5)
    cfg = n2f.default_config(fixed_epochs=6)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=2)
    assert b.run(max_epochs=2) == 2           # two images still training after 2 epochs each
    assert b.run() == 0
    assert torch.equal(b.result(1).cpu(), torch.from_numpy(imgs[1]))
    ya, _ = n2f.denoise(dev(imgs[2]), cfg)
    assert torch.equal(b.result(2), ya)


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_server_results_equal_alone(prec):
    """Requests arrive while others train; the arena holds only a few runs at
    a time, so later requests wait for memory and join as others leave."""
    shapes = SHAPES + [(1, 70, 90), (3, 36, 30), (1, 128, 64)]
    imgs = _images(shapes, seed=10)
    cfg = n2f.default_config(precision=prec, patience=4, max_epochs=50)
    arena = 3 * max(n2f.workspace_bytes(H, W, C, cfg) for C, H, W in shapes)
    srv = n2f.Server(arena, cfg, n_streams=3, max_active=8)
    xs = [dev(x) for x in imgs]
    outs = [torch.empty_like(x) for x in xs]
    pending = list(range(len(xs)))
    finished = {}
    steps = 0
    while len(finished) < len(xs):
        # two new arrivals every scheduling round
        for _ in range(2):
            if pending:
                i = pending.pop(0)
                srv.submit(i, xs[i], outs[i])
        active, queued = srv.step(2)
        used, largest = srv.memory()
        assert used <= arena
        for rid, st in srv.poll():
            assert st in (n2f.OK, n2f.WCAPPED)
            finished[rid] = steps
        steps += 1
        assert steps < 500
    for i, x in enumerate(xs):
        ya, _ = n2f.denoise(x, cfg)
        assert torch.equal(outs[i], ya), i
    assert srv.memory() == (0, arena)
