"""Failure handling, forced from the host so that every kernel still runs
normally: a non-finite validation score (a NaN head bias loaded through the
state-exchange calls) ends that network with N2F_ENUMERIC; in a batch only
that image fails; in the server a request with a non-finite input fails
alone and the others match their runs alone."""
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


def scene(C, H, W, seed):
    return synth.add_gaussian(synth.blobs(H, W, seed, C=C), 25 / 255, seed + 50)


def poison(run, net=0):
    """Load a NaN head bias (the last canonical parameter) into one network."""
    th, m, v, t = run.get_state(net)
    th[-1] = np.nan
    run.set_state(net, th, m, v, t)


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_nonfinite_score_ends_the_network(prec):
    say("nonfinite single", prec)
    cfg = n2f.default_config(precision=prec, patience=5, max_epochs=40)
    x = dev(scene(1, 40, 36, 1))
    r = n2f.Run(x, cfg)
    poison(r)
    with pytest.raises(n2f.N2FError) as e:
        r.validate(0)
    assert e.value.code == n2f.ENUMERIC
    assert r.progress(0)[0] == 1 and np.isnan(r.history(0)[0])
    with pytest.raises(n2f.N2FError) as e:
        r.train_step(0, 0)
    assert e.value.code == n2f.ESTATE
    # the queued-epochs path (graph replay) stops after the same epoch
    r2 = n2f.Run(x, cfg)
    poison(r2)
    with pytest.raises(n2f.N2FError) as e:
        r2.run_epochs(0, 40)
    assert e.value.code == n2f.ENUMERIC
    assert r2.progress(0)[0] == 1


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_batch_image_fails_alone(prec):
    say("nonfinite batch", prec)
    cfg = n2f.default_config(precision=prec, fixed_epochs=4)
    imgs = [scene(1, 40, 36, 2), scene(3, 30, 34, 3), scene(1, 52, 44, 4)]
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=2)
    poison(b.run_of(1), net=1)          # the second network of the RGB image
    assert b.run() == 0
    with pytest.raises(n2f.N2FError) as e:
        b.result(1)
    assert e.value.code == n2f.ENUMERIC
    assert b.progress(1)[1]
    for i in (0, 2):
        ya, _ = n2f.denoise(dev(imgs[i]), cfg)
        assert torch.equal(b.result(i), ya), i


def test_server_request_with_nonfinite_input_fails_alone():
    say("nonfinite server")
    cfg = n2f.default_config(precision=n2f.BF16, fixed_epochs=3)
    imgs = [scene(1, 40, 36, 5), scene(1, 33, 47, 6), scene(3, 24, 30, 7)]
    bad = imgs[1].copy()
    bad[0, 4, 5] = np.inf
    imgs[1] = bad
    arena = 4 * max(n2f.workspace_bytes(x.shape[1], x.shape[2], x.shape[0], cfg) for x in imgs)
    srv = n2f.Server(arena, cfg, n_streams=2, max_active=4)
    xs = [dev(x) for x in imgs]
    outs = [torch.zeros_like(x) for x in xs]
    for i, x in enumerate(xs):
        srv.submit(i, x, outs[i])
    status = {}
    for _ in range(50):
        srv.step(1)
        for rid, st in srv.poll():
            status[rid] = st
        if len(status) == len(xs):
            break
    assert status == {0: n2f.OK, 1: n2f.EINVAL, 2: n2f.OK}
    assert srv.memory()[0] == 0
    for i in (0, 2):
        ya, _ = n2f.denoise(xs[i], cfg)
        assert torch.equal(outs[i], ya), i
