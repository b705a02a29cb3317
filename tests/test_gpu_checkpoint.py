"""Whole-network checkpoints: a run saved part way and resumed in a fresh
run from the same image and configuration finishes bit-identically to the
run left alone (same output, stopping epoch, best epoch and validation
history); blobs from another image size or configuration are refused."""
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
    return synth.add_gaussian(synth.blobs(H, W, seed, C=C), 25 / 255, seed + 70)


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
@pytest.mark.parametrize("C,phase", [(1, "mid"), (3, "mid"), (3, "later")])
def test_resume_is_bit_identical(prec, C, phase):
    """mid: network 0 saved after 5 epochs (the others untouched); later:
    network 0 finished and network 1 saved after 5 epochs."""
    say("checkpoint", prec, C, phase)
    x = dev(scene(C, 44, 52, 11))
    cfg = n2f.default_config(precision=prec, patience=8, max_epochs=300)
    a = n2f.Run(x, cfg)
    if phase == "mid":
        a.run_epochs(0, 5)
    else:
        a.run_epochs(0, 300)
        a.run_epochs(1, 5)
    cks = [a.save_checkpoint(k) for k in range(C)]
    saved = [a.progress(k) for k in range(C)]
    assert saved[0 if phase == "mid" else 1][0] == 5
    for k in range(C):
        a.run_epochs(k, 300)
    ya = a.result()
    b = n2f.Run(x, cfg)
    for k in range(C):
        b.load_checkpoint(k, cks[k])
        assert b.progress(k) == saved[k]
    for k in range(C):
        b.run_epochs(k, 300)
    yb = b.result()
    assert torch.equal(ya, yb)
    for k in range(C):
        assert a.progress(k) == b.progress(k)
        np.testing.assert_array_equal(a.history(k), b.history(k))


def test_checkpoint_mismatch_is_refused():
    x = dev(scene(1, 40, 40, 12))
    a = n2f.Run(x, n2f.default_config())
    ck = a.save_checkpoint(0)
    for other in (n2f.Run(dev(scene(1, 40, 42, 13)), n2f.default_config()),
                  n2f.Run(x, n2f.default_config(precision=n2f.BF16)),
                  n2f.Run(x, n2f.default_config(downsample=n2f.DS_QUAD))):
        with pytest.raises(n2f.N2FError) as e:
            other.load_checkpoint(0, ck)
        assert e.value.code == n2f.EINVAL
    with pytest.raises(n2f.N2FError) as e:
        a.load_checkpoint(0, ck[:-1])
    assert e.value.code == n2f.EINVAL
    bad = ck.copy()
    bad[0] ^= 0xFF
    with pytest.raises(n2f.N2FError) as e:
        a.load_checkpoint(0, bad)
    assert e.value.code == n2f.EINVAL
    a.load_checkpoint(0, ck)
