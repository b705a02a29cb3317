"""Grouped batches (n_streams = BATCH_GROUPED): every launch of an epoch is
one launch over all images of the same channel count, whose blocks run each
image's blocks exactly as the image's own launch would.  Each image's result,
stopping epoch and validation history must therefore be the same bits as the
image denoised alone, whatever else is in the group, and images may join,
leave, fail or move on to their next network at epoch boundaries."""
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


def _images(shapes, seed=0):
    out = []
    for i, (C, H, W) in enumerate(shapes):
        clean = synth.blobs(H, W, seed + i, C=C)
        out.append(synth.add_gaussian(clean, 25 / 255, seed + 50 + i))
    return out


# mixed sizes (odd, non-square, tiny and multi-tile), one to three channels
SHAPES = [(1, 96, 80), (1, 64, 130), (3, 40, 44), (1, 121, 72), (2, 33, 35), (1, 2, 3), (1, 300, 170),
          (3, 24, 20), (1, 50, 66)]


def _alone(x, cfg):
    r = n2f.Run(dev(x), cfg)
    C = x.shape[0]
    for k in range(C):
        done, status = r.run_epochs(k, 100000)
        assert done
    return r.result(), [r.progress(k) for k in range(C)], [r.history(k) for k in range(C)]


@pytest.mark.parametrize("kw,streams", [(dict(fixed_epochs=4), n2f.BATCH_GROUPED),
                                        (dict(patience=4, max_epochs=60), n2f.BATCH_GROUPED),
                                        (dict(patience=3, max_epochs=40, downsample=n2f.DS_QUAD), n2f.BATCH_GROUPED),
                                        (dict(patience=4, max_epochs=60), -2), (dict(fixed_epochs=4), -3),
                                        (dict(fixed_epochs=4, wgrad_splits=8), n2f.BATCH_GROUPED)])
def test_grouped_batch_equals_alone(kw, streams):
    """On the caller's stream (-1) or split over 2 or 3 streams of the
    batch's own (-2, -3): every image ends as it would alone."""
    say("grouped batch", kw, streams)
    imgs = _images(SHAPES)
    cfg = n2f.default_config(precision=n2f.BF16, **kw)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=streams)
    assert b.run() == 0
    for i, x in enumerate(imgs):
        yb = b.result(i)
        ya, prog, hist = _alone(x, cfg)
        assert torch.equal(yb, ya), i
        rb = b.run_of(i)
        for k in range(x.shape[0]):
            assert rb.progress(k) == prog[k], (i, k)
            np.testing.assert_array_equal(rb.history(k), hist[k])
        assert b.progress(i)[1]
    b.close()


def test_grouped_multi_tile_image_equals_alone():
    """A 768x768 image (training images of 1152 tiles: several tiles per
    block, several splits per weight-gradient block) next to small ones."""
    say("grouped 768")
    imgs = _images([(1, 768, 768), (1, 70, 90), (1, 257, 129)], seed=7)
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=3)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=n2f.BATCH_GROUPED)
    assert b.run() == 0
    for i, x in enumerate(imgs):
        assert torch.equal(b.result(i), _alone(x, cfg)[0]), i
    b.close()


@pytest.mark.parametrize("streams", [n2f.BATCH_GROUPED, -2])
def test_grouped_add_remove_and_partial_runs(streams):
    """Runs of a few epochs at a time; an image joins mid-way, another leaves;
    the ones that stay and the one that joins end as they would alone."""
    say("grouped add/remove", streams)
    imgs = _images([(1, 60, 52), (1, 45, 80), (3, 30, 26), (1, 90, 40)], seed=20)
    cfg = n2f.default_config(precision=n2f.BF16, patience=3, max_epochs=50)
    b = n2f.Batch([dev(x) for x in imgs[:3]], cfg, n_streams=streams)
    assert b.run(max_epochs=2) > 0
    b.remove(1)
    j = b.add(dev(imgs[3]))
    assert j == 3
    assert b.run() == 0
    for i in (0, 2, 3):
        assert torch.equal(b.result(i), _alone(imgs[i], cfg)[0]), i
    with pytest.raises(n2f.N2FError) as e:
        b.result(1)
    assert e.value.code == n2f.ESTATE
    b.close()


def test_grouped_failure_is_isolated():
    """A NaN head bias loaded into one image's network makes its score
    non-finite: that image fails alone (ENUMERIC), the others are unchanged."""
    say("grouped failure")
    imgs = _images([(1, 40, 48), (1, 36, 50), (1, 52, 30)], seed=30)
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=5)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=n2f.BATCH_GROUPED)
    r1 = b.run_of(1)
    th, m, v, t = r1.get_state(0)
    th[-1] = np.nan
    r1.set_state(0, th, m, v, t)
    assert b.run() == 0
    with pytest.raises(n2f.N2FError) as e:
        b.result(1)
    assert e.value.code == n2f.ENUMERIC
    for i in (0, 2):
        assert torch.equal(b.result(i), _alone(imgs[i], cfg)[0]), i
    b.close()


def test_grouped_kernel_timing_classes():
    """The profiler times every grouped launch by kind; the 3x3 kinds count
    the pixels of every image they cover."""
    imgs = _images([(1, 64, 64), (1, 48, 80)], seed=40)
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=2)
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=n2f.BATCH_GROUPED)
    n2f.profile_begin(1)
    b.run()
    n2f.profile_end()
    ms, n, px = n2f.profile_read(n2f.K_GROUP + 0)     # plain forward: 5 per training step, 5 per validation
    assert n == 2 * (4 * 5 + 5) and ms > 0
    assert px == 2 * (4 * 5 * (64 * 32) + 5 * (64 * 64)) + 2 * (2 * 5 * (48 * 40) + 2 * 5 * (24 * 80) + 5 * 48 * 80)
    b.close()


def test_grouped_server_results_equal_alone():
    """Grouped serving (N2F_SERVER_GROUPED): requests of one and three
    channels arrive while others train, wait for arena space, join their
    channel count's group and leave it at epoch boundaries; each result is
    the same bits as the request denoised alone."""
    say("grouped server")
    shapes = SHAPES + [(1, 70, 90), (3, 36, 30), (1, 128, 64)]
    imgs = _images(shapes, seed=60)
    cfg = n2f.default_config(precision=n2f.BF16, patience=4, max_epochs=50)
    arena = 3 * max(n2f.workspace_bytes(H, W, C, cfg) for C, H, W in shapes)
    srv = n2f.Server(arena, cfg, max_active=8, grouped=True)
    xs = [dev(x) for x in imgs]
    outs = [torch.empty_like(x) for x in xs]
    pending = list(range(len(xs)))
    finished, steps = {}, 0
    while len(finished) < len(xs):
        for _ in range(2):
            if pending:
                i = pending.pop(0)
                srv.submit(i, xs[i], outs[i])
        srv.step(2)
        for rid, st in srv.poll():
            assert st in (n2f.OK, n2f.WCAPPED)
            finished[rid] = steps
        steps += 1
        assert steps < 500
    for i, x in enumerate(imgs):
        assert torch.equal(outs[i], _alone(x, cfg)[0]), i
    srv.close()


def test_launch_geometry_never_changes_results():
    """Other grids for the grouped kinds (fewer and more hardware blocks than
    virtual blocks) give the same bits; the tuner's entry covers every kind
    it timed and leaves valid grids."""
    say("group grids")
    imgs = _images([(1, 96, 80), (3, 40, 44), (1, 300, 170), (1, 50, 66)], seed=70)
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=3)
    saved = [n2f.group_grid(k) for k in range(len(n2f.GROUP_KINDS))]
    try:
        ref = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=n2f.BATCH_GROUPED)
        assert ref.run() == 0
        for grid in (1, 7, 1024):
            for k in range(len(n2f.GROUP_KINDS)):
                n2f.set_group_grid(k, grid)
            b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=n2f.BATCH_GROUPED)
            assert b.run() == 0
            for i in range(len(imgs)):
                assert torch.equal(b.result(i), ref.result(i)), (grid, i)
            b.close()
        ref.close()
        for k, g in enumerate(saved):
            n2f.set_group_grid(k, g)
        from paper_2108_10209_amd import autotune
        entry = autotune.tune([dev(x) for x in imgs[:2]], candidates=(64, 512), epochs=1, log=lambda *a: None)
        assert "conv3x3_wgrad" in entry["group_grid"] and "adam" in entry["group_grid"]
        for name, g in entry["group_grid"].items():
            assert g in (64, 512, saved[n2f.GROUP_KINDS.index(name)])
            assert n2f.group_grid(n2f.GROUP_KINDS.index(name)) == g
    finally:
        for k, g in enumerate(saved):
            n2f.set_group_grid(k, g)
