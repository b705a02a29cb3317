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


@pytest.mark.parametrize("n_streams", [0, 2])
def test_batch_add_and_remove_at_epoch_boundaries(n_streams):
    """Images join and leave between batch runs (epoch boundaries): the
    images that stay, and the one that joins, end with the same bits as
    when denoised alone; a removed image's calls are refused.  n_streams = 0
    runs the whole batch on the caller's stream."""
    say("batch add/remove", n_streams)
    imgs = _images(SHAPES[:3] + [(1, 72, 58)], seed=30)
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=6)
    b = n2f.Batch([dev(x) for x in imgs[:3]], cfg, n_streams=n_streams)
    assert b.run(max_epochs=2) == 3
    j = b.add(dev(imgs[3]))
    assert j == 3
    b.remove(1)
    with pytest.raises(n2f.N2FError) as e:
        b.result(1)
    assert e.value.code == n2f.ESTATE
    with pytest.raises(n2f.N2FError):
        b.remove(1)
    assert b.progress(1)[1]
    assert b.run() == 0
    for i in (0, 2, 3):
        ya, _ = n2f.denoise(dev(imgs[i]), cfg)
        assert torch.equal(b.result(i), ya), i
    b.close()


def test_batch_reads_inputs_after_the_callers_stream():
    """Inputs produced on the caller's (non-default) stream just before the
    batch is created, with no host synchronisation: the batch's streams wait
    for that stream, so the results equal the images denoised alone."""
    imgs = _images(SHAPES[:3], seed=40)
    cfg = n2f.default_config(fixed_epochs=3)
    side = torch.cuda.Stream(DEV)
    with torch.cuda.stream(side):
        base = [dev(x) for x in imgs]
        side.synchronize()
        # a chain of device work on the caller's stream that produces the inputs
        xs = [(x * 3.0 - 1.0).add_(1.0).div_(3.0) for x in base]
        b = n2f.Batch(xs, cfg, n_streams=2)
    assert b.run() == 0
    torch.cuda.synchronize()
    for i, x in enumerate(xs):
        ya, _ = n2f.denoise(x, cfg)
        assert torch.equal(b.result(i), ya), i


def test_server_cancel_on_device():
    """A cancelled request (active or still queued) leaves the arena at once,
    its output buffer is never written, and the other requests still end
    with the same bits as alone."""
    cfg = n2f.default_config(precision=n2f.BF16, patience=4, max_epochs=40)
    imgs = _images([(1, 64, 64), (1, 80, 72), (1, 70, 66), (1, 60, 90)], seed=60)
    arena = 2 * max(n2f.workspace_bytes(H, W, C, cfg) for C, H, W in [x.shape for x in imgs])
    srv = n2f.Server(arena, cfg, n_streams=2, max_active=2)
    xs = [dev(x) for x in imgs]
    outs = [torch.full_like(x, float("nan")) for x in xs]
    for i in range(4):
        srv.submit(i, xs[i], outs[i])
    srv.step(2)                     # 0 and 1 active, 2 and 3 queued
    srv.cancel(1)
    srv.cancel(3)
    rep = dict(srv.poll())
    assert rep == {1: n2f.ECANCELED, 3: n2f.ECANCELED}
    for _ in range(200):
        srv.step(2)
        rep.update(srv.poll())
        if len(rep) == 4:
            break
    assert rep[0] in (n2f.OK, n2f.WCAPPED) and rep[2] in (n2f.OK, n2f.WCAPPED)
    torch.cuda.synchronize()
    assert torch.isnan(outs[1]).all() and torch.isnan(outs[3]).all()
    for i in (0, 2):
        ya, _ = n2f.denoise(xs[i], cfg)
        assert torch.equal(outs[i], ya), i
    assert srv.memory() == (0, arena)


def test_served_results_match_the_oracle():
    """Served requests (grayscale and RGB, uneven sizes, arriving while
    others train) against the CPU FP64 oracle run on each image alone:
    FP32, 3 fixed epochs, every output within 1e-4 (norm-wise)."""
    from oracle import n2f_oracle as O
    shapes = [(1, 48, 40), (3, 36, 30), (1, 33, 52), (3, 24, 28)]
    imgs = _images(shapes, seed=70)
    cfg = n2f.default_config(fixed_epochs=3)
    arena = 2 * max(n2f.workspace_bytes(H, W, C, cfg) for C, H, W in shapes)
    srv = n2f.Server(arena, cfg, n_streams=2, max_active=4)
    xs = [dev(x) for x in imgs]
    outs = [torch.empty_like(x) for x in xs]
    done, nxt = {}, 0
    for _ in range(200):
        if nxt < len(xs):
            srv.submit(nxt, xs[nxt], outs[nxt])
            nxt += 1
        srv.step(1)
        done.update(srv.poll())
        if len(done) == len(xs):
            break
    assert all(st == n2f.OK for st in done.values()) and len(done) == len(xs)
    for i, (C, H, W) in enumerate(shapes):
        ref = O.denoise(imgs[i].astype(np.float64), synth.init_params(C, 0), O.Hyper(fixed_epochs=3))
        y = outs[i].cpu().numpy()
        err = float(np.linalg.norm(y - ref.y) / np.linalg.norm(ref.y))
        say("served", i, (C, H, W), "rel err vs oracle", err)
        assert err < 1e-4, (i, err)


@pytest.mark.parametrize("n_streams,max_active", [(2, 2), (1, 4)])
def test_served_results_match_oracle(n_streams, max_active):
    """FP32 requests served in a mix (grayscale and RGB, uneven sizes, a few
    admitted at a time so later ones join as earlier ones leave) against the
    CPU FP64 oracle run on each request alone from the same initial weights,
    three fixed epochs: every output channel within 1e-4 norm-wise.  (With
    the stopping rule on, the stopping epoch of a tiny image can move with
    rounding; the stopping rule is checked step by step elsewhere.)"""
    from oracle import n2f_oracle as O
    kw = dict(fixed_epochs=3)
    shapes = [(1, 40, 48), (3, 24, 20), (1, 33, 50), (1, 64, 30)]
    imgs = _images(shapes, seed=40)
    cfg = n2f.default_config(**kw)
    arena = max_active * max(n2f.workspace_bytes(H, W, C, cfg) for C, H, W in shapes)
    srv = n2f.Server(arena, cfg, n_streams=n_streams, max_active=max_active)
    xs = [dev(x) for x in imgs]
    outs = [torch.empty_like(x) for x in xs]
    for i in range(len(xs)):
        srv.submit(i, xs[i], outs[i])
    done, steps = {}, 0
    while len(done) < len(xs):
        srv.step(1)
        done.update(dict(srv.poll()))
        steps += 1
        assert steps < 1000
    hyp = O.Hyper(fixed_epochs=3)
    for i, (x, (C, H, W)) in enumerate(zip(imgs, shapes)):
        assert done[i] == n2f.OK, (i, done[i])
        ref = O.denoise(x, synth.init_params(C, 0), hyp)
        y = outs[i].cpu().numpy()
        for k in range(C):
            err = float(np.linalg.norm(y[k] - ref.y[k]) / np.linalg.norm(ref.y[k]))
            say(f"  request {i} ({C}x{H}x{W}) channel {k}: rel err {err:.2e}, epochs {ref.epochs[k]}")
            assert err < 1e-4, (i, k, err)
