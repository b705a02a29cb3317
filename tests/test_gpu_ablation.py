"""Ablations of the Noise2Fast study (Methods, Ablation Study; Table 1) on
the GPU against the CPU FP64 oracle, through the C ABI: 2x2-block ("Quad")
downsampling and "Exact" targets.  Same bars as the main path: downsamples
bit-exact; Exact targets within a few FP32 ulps of their FP64 value; a
teacher-forced step within norm-wise relative error 1e-5 (FP32) or 2e-2
(BF16) per tensor; fixed-epoch PSNR within 0.1 dB of the oracle's.  A BF16
tensor that BF16 rounding alone moves by more than 1e-2 (ill-conditioned) may
instead match a model of the path's rounding within 2e-2 (see `bf16_bar`)."""
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


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def split(vec, C):
    out, o = {}, 0
    for name, shape in O.param_spec(C):
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n])
        o += n
    return out


def library_order(tl, tr, bl, br):
    """The library keeps the 2x2-block images so that pair p trains image p:
    TL, BR, TR, BL."""
    return [tl, br, tr, bl]


def scene(C, H, W, seed):
    clean = synth.blobs(H, W, seed, C=C)
    return clean, synth.add_gaussian(clean, 25 / 255, seed + 100)


def step_errors(r, C, k, st, pairs, pair):
    """Load the oracle state st into network k, run one GPU step on `pair`
    and return the per-tensor gradient errors and the loss error against the
    oracle's step from the FP32-rounded state, and the GPU gradient."""
    r.set_state(k, st.theta, st.m, st.v, st.t)
    st32 = O.NetState(st.theta.astype(np.float32).astype(np.float64), st.m.astype(np.float32).astype(np.float64),
                      st.v.astype(np.float32).astype(np.float64), st.t)
    r.train_step(k, pair)
    g, loss = r.get_grad(k)
    inp, tgt = pairs[pair]
    _, g_or, loss_or, _ = O.train_step(st32, C, inp, tgt[k], H0)
    errs = {nm: rel(a, b) for (nm, a), b in zip(split(g, C).items(), split(g_or, C).values())}
    return errs, abs(loss - loss_or) / abs(loss_or), g


# ---------------------------------------------------------------------------
# 2x2-block downsampling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("C,H,W", [(1, 64, 64), (1, 37, 50), (3, 33, 17), (1, 2, 2), (3, 130, 96), (1, 512, 512)])
def test_quad_prepare_bit_exact(C, H, W):
    say("quad prepare", C, H, W)
    rng = np.random.default_rng(H * W + C + 1)
    x = (rng.standard_normal((C, H, W)) * 2 + 1).astype(np.float32)
    r = n2f.Run(dev(x), n2f.default_config(downsample=n2f.DS_QUAD))
    xs = r.image(4).cpu().numpy()
    xs_or, _, _ = O.standardize(x)
    ulp = np.abs(xs.view(np.int32).astype(np.int64) - xs_or.astype(np.float32).view(np.int32).astype(np.int64))
    assert ulp.max() <= 1
    refs = library_order(*O.quad_downsample(xs.astype(np.float64)))
    for which, ref in enumerate(refs):
        got = r.image(which).cpu().numpy()
        assert got.shape == ref.shape == (C, H // 2, W // 2)
        np.testing.assert_array_equal(got, ref.astype(np.float32))
        # without exact targets, pair p's target is its partner image
        np.testing.assert_array_equal(r.image(8 + which).cpu().numpy(), refs[[1, 0, 3, 2][which]].astype(np.float32))


@pytest.mark.parametrize("C,H,W", [(1, 16, 16), (2, 9, 14), (3, 64, 62)])
def test_quad_index_image(C, H, W):
    """On the index image every block image pixel names its source pixel."""
    say("quad index", C, H, W)
    x = synth.index_image(C, H, W)
    r = n2f.Run(dev(x), n2f.default_config(downsample=n2f.DS_QUAD))
    n = C * H * W - 1
    for which, ref in enumerate(library_order(*O.quad_downsample(x.astype(np.float64)))):
        got = np.rint(r.image(which).cpu().numpy().astype(np.float64) * n)
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("prec,C,H,W,pre", [
    (n2f.FP32, 1, 64, 64, 0), (n2f.FP32, 1, 64, 64, 5), (n2f.FP32, 3, 40, 36, 3), (n2f.FP32, 1, 33, 97, 1),
    (n2f.FP32, 1, 130, 66, 2),
    (n2f.BF16, 1, 64, 64, 6), (n2f.BF16, 3, 36, 40, 2), (n2f.BF16, 1, 512, 512, 1),
])
def test_quad_train_step_teacher_forced(prec, C, H, W, pre):
    say("quad step", prec, C, H, W, pre)
    _, noisy = scene(C, H, W, 2)
    r = n2f.Run(dev(noisy), n2f.default_config(downsample=n2f.DS_QUAD, precision=prec))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    pairs = O.training_pairs(xs, "quad")
    for k in range(C):
        st = O.new_state(th0[k])
        for s in range(pre):
            st = O.train_step(st, C, pairs[s % 4][0], pairs[s % 4][1][k], H0)[0]
        errs, lerr, g = step_errors(r, C, k, st, pairs, pre % 4)
        if prec == n2f.FP32:
            worst = max(errs, key=errs.get)
            say("  worst grad err", worst, errs[worst], "loss err", lerr)
            assert all(e < 1e-5 for e in errs.values()), errs
        else:
            inp, tgt = pairs[pre % 4]
            ok, rows = bf16_check(g, st.theta.astype(np.float32).astype(np.float64), C, inp, tgt[k])
            say("  " + summary(rows), "loss err", lerr)
            assert ok, rows
        assert lerr < (1e-6 if prec == n2f.FP32 else 2e-2)


def test_quad_small_64_fixed_8_epochs():
    """64x64, sigma 25/255, 8 fixed epochs with 2x2 blocks: free-running PSNR
    within 0.1 dB of the oracle's, validation scores within 1e-3."""
    say("quad 64x64 8 epochs")
    clean, noisy = synth.small_64(0)
    th0 = synth.init_params(1, 0)
    cfg = n2f.default_config(fixed_epochs=8, downsample=n2f.DS_QUAD)
    r = n2f.Run(dev(noisy), cfg)
    done, status = r.run_epochs(0, 8)
    assert done and status == n2f.OK
    y = r.result().cpu().numpy()
    ref = O.denoise(noisy, th0, O.Hyper(fixed_epochs=8), downsample="quad")
    p_gpu, p_or = synth.psnr(y, clean), synth.psnr(ref.y, clean)
    say("psnr gpu", p_gpu, "oracle", p_or, "noisy", synth.psnr(noisy, clean))
    assert abs(p_gpu - p_or) < 0.1
    np.testing.assert_allclose(r.history(0), ref.history[0], rtol=1e-3)
    y1, st1 = n2f.denoise(dev(noisy), cfg)
    assert st1 == n2f.OK and torch.equal(y1.cpu(), torch.from_numpy(y))


def test_quad_batch_equals_alone():
    """Batched 2x2-block runs give the same bits as the same runs alone."""
    say("quad batch")
    cfg = n2f.default_config(fixed_epochs=3, downsample=n2f.DS_QUAD, precision=n2f.BF16)
    imgs = [scene(1, 48, 40, 30)[1], scene(3, 34, 52, 31)[1], scene(1, 70, 66, 32)[1]]
    b = n2f.Batch([dev(x) for x in imgs], cfg, n_streams=2)
    b.run()
    for i, x in enumerate(imgs):
        ya, _ = n2f.denoise(dev(x), cfg)
        assert torch.equal(b.result(i).cpu(), ya.cpu()), i


# ---------------------------------------------------------------------------
# "Exact" targets
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ds,C,H,W", [("checkerboard", 1, 64, 64), ("checkerboard", 3, 33, 17),
                                      ("quad", 1, 37, 50), ("quad", 3, 130, 96), ("checkerboard", 1, 512, 512)])
def test_exact_targets_match_oracle(ds, C, H, W):
    """Targets x_b - (s_b - s_a) in FP32 against the FP64 value: a few ulps
    of the target's scale (three roundings plus the standardisation's)."""
    say("exact targets", ds, C, H, W)
    clean, noisy = scene(C, H, W, 3)
    cfg = n2f.default_config(exact_targets=1, downsample=n2f.DS_QUAD if ds == "quad" else n2f.DS_CHECKERBOARD)
    r = n2f.Run(dev(noisy), cfg)
    with pytest.raises(n2f.N2FError) as e:
        r.train_step(0, 0)
    assert e.value.code == n2f.ESTATE
    r.set_clean(dev(clean))
    x_std, lo, hi = O.standardize(noisy)
    pairs = O.exact_pairs(x_std, (clean.astype(np.float64) - lo) / (hi - lo), ds)
    for p, (_, tgt) in enumerate(pairs):
        got = r.image(8 + p).cpu().numpy().astype(np.float64)
        assert got.shape == tgt.shape
        err = np.abs(got - tgt).max()
        assert err <= 8 * np.finfo(np.float32).eps * max(1.0, np.abs(tgt).max()), (p, err)


def test_exact_clean_image_errors_and_replacement():
    clean, noisy = scene(1, 24, 20, 4)
    r = n2f.Run(dev(noisy), n2f.default_config(exact_targets=1))
    bad = clean.copy()
    bad[0, 5, 6] = np.inf
    with pytest.raises(n2f.N2FError) as e:
        r.set_clean(dev(bad))
    assert e.value.code == n2f.EINVAL
    with pytest.raises(n2f.N2FError) as e:
        r.run_epochs(0, 1)
    assert e.value.code == n2f.ESTATE
    with pytest.raises(n2f.N2FError) as e:
        r.image(8)
    assert e.value.code == n2f.ESTATE
    # a clean image equal to the noisy one makes every target its input
    r.set_clean(dev(noisy))
    for p in range(4):
        np.testing.assert_allclose(r.image(8 + p).cpu().numpy(), r.image(p).cpu().numpy(), rtol=0, atol=1e-6)
    r.set_clean(dev(clean))
    r.train_step(0, 0)
    plain = n2f.Run(dev(noisy))
    with pytest.raises(n2f.N2FError) as e:
        plain.set_clean(dev(clean))
    assert e.value.code == n2f.ESTATE


@pytest.mark.parametrize("ds", ["checkerboard", "quad"])
def test_exact_teacher_forced_and_fixed_epochs(ds):
    """64x64 scene: a teacher-forced step on Exact targets within 1e-5, and
    8 free-running epochs within 0.1 dB of the oracle's PSNR."""
    say("exact 64x64", ds)
    clean, noisy = synth.small_64(0)
    th0 = synth.init_params(1, 0)
    mode = n2f.DS_QUAD if ds == "quad" else n2f.DS_CHECKERBOARD
    cfg = n2f.default_config(fixed_epochs=8, exact_targets=1, downsample=mode)
    r = n2f.Run(dev(noisy), cfg)
    r.set_clean(dev(clean))
    x_std, lo, hi = O.standardize(noisy)
    pairs = O.exact_pairs(x_std, (clean.astype(np.float64) - lo) / (hi - lo), ds)
    st = O.new_state(th0[0])
    for s in range(3):
        st = O.train_step(st, 1, pairs[s][0], pairs[s][1][0], H0)[0]
    errs, lerr, _ = step_errors(r, 1, 0, st, pairs, 3)
    say("  worst grad err", max(errs.values()), "loss err", lerr)
    assert max(errs.values()) < 1e-5 and lerr < 1e-6
    r2 = n2f.Run(dev(noisy), cfg)
    r2.set_clean(dev(clean))
    done, status = r2.run_epochs(0, 8)
    assert done and status == n2f.OK
    y = r2.result().cpu().numpy()
    ref = O.denoise(noisy, th0, O.Hyper(fixed_epochs=8), downsample=ds, clean=clean)
    p_gpu, p_or = synth.psnr(y, clean), synth.psnr(ref.y, clean)
    say("psnr gpu", p_gpu, "oracle", p_or, "noisy", synth.psnr(noisy, clean))
    assert abs(p_gpu - p_or) < 0.1
