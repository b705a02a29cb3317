"""Volumes (Methods, Fluorescence Microscopy Images): z-slices denoised one
by one, then max projected.  The projection kernel is bit-exact against the
oracle's; slices denoised in one batch are bit-identical to the same slices
denoised alone; the FP32 slices and their projection agree with the FP64
oracle after fixed epochs."""
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("Z,H,W,offset", [(41, 64, 64, 0), (1, 5, 7, 0), (3, 33, 17, 0), (7, 1024, 1024, 0),
                                          (5, 16, 16, 1), (2, 1, 3, 0), (41, 1024, 1024, 0)])
def test_max_project_bit_exact(Z, H, W, offset):
    """Vector path (pixel count a multiple of 4, aligned) and scalar path
    (ragged count, or a stack starting one float past an aligned address)."""
    say("max project", Z, H, W, offset)
    rng = np.random.default_rng(Z + H + W + offset)
    st = rng.standard_normal((Z, H, W)).astype(np.float32)
    if H * W >= 4:
        st[:, 0, 1] = np.nan               # all-NaN column stays NaN
        st[0, 0, 2] = np.nan               # a NaN loses to any number
    buf = torch.empty(Z * H * W + offset, dtype=torch.float32, device=DEV)
    stack = buf[offset:].view(Z, H, W)
    stack.copy_(torch.from_numpy(st))
    got = n2f.max_project(stack).cpu().numpy()
    ref = O.max_projection(st.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(got, ref)


def test_max_project_rejects_overlap():
    st = torch.zeros((3, 8, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(n2f.N2FError) as e:
        n2f.max_project(st, out=st[1])
    assert e.value.code == n2f.EINVAL


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_volume_batch_slices_and_projection(prec):
    """A 4-slice stack (one channel of a synthetic cell volume) denoised as
    one batch: each slice bit-identical to it denoised alone, the projection
    bit-identical to the oracle's projection of those slices; in FP32 the
    slices and the projection within 1e-4 of the FP64 oracle's."""
    say("volume", prec)
    Z, H, W = 4, 40, 48
    clean = synth.cell_volume(Z, H, W, seed=9)[0]
    noisy = synth.add_poisson_gaussian(clean, 10.0, 0.02, 19)
    cfg = n2f.default_config(fixed_epochs=2, precision=prec)
    xs = [torch.from_numpy(np.ascontiguousarray(noisy[z][None])).to(DEV) for z in range(Z)]
    b = n2f.Batch(xs, cfg, n_streams=2)
    b.run()
    den = torch.stack([b.result(i)[0] for i in range(Z)]).contiguous()
    b.close()
    for z in range(Z):
        alone, _ = n2f.denoise(xs[z], cfg)
        assert torch.equal(alone[0].cpu(), den[z].cpu()), z
    proj = n2f.max_project(den).cpu().numpy()
    den_np = den.cpu().numpy()
    np.testing.assert_array_equal(proj, O.max_projection(den_np.astype(np.float64)).astype(np.float32))
    if prec == n2f.FP32:
        ref_proj, ref_den = O.denoise_volume(noisy.astype(np.float64), synth.init_params(1, 0),
                                             O.Hyper(fixed_epochs=2))
        for z in range(Z):
            assert rel(den_np[z], ref_den[z]) < 1e-4, z
        assert rel(proj, ref_proj) < 1e-4
