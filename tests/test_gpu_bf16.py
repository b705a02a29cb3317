"""BF16 convolution path (BF16 operands on the MFMA, FP32 accumulation, FP32
master weights and Adam, FP64 validation sum) against the FP64 oracle and
against the GPU FP32 path.  Bars: teacher-forced step within norm-wise
relative error 2e-2 per tensor; final PSNR within 0.1 dB of FP32."""
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H0 = O.Hyper()
TOL = 2e-2


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


def bf16_cfg(**kw):
    return n2f.default_config(precision=n2f.BF16, **kw)


# 512x512 is the benchmark's image size, in the launch configuration it times
@pytest.mark.parametrize("C,H,W", [(1, 64, 64), (3, 40, 33), (1, 45, 70), (1, 512, 512)])
def test_bf16_validation_forward(C, H, W):
    say("bf16 validate", C, H, W)
    clean = synth.blobs(H, W, 1, C=C)
    noisy = synth.add_gaussian(clean, 25 / 255, 11)
    r = n2f.Run(dev(noisy), bf16_cfg())
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    for k in range(C):
        v, imp, _ = r.validate(k)
        y = r.image(5 + k).cpu().numpy()
        y_or, v_or = O.validate(th0[k], C, xs, k, H0)
        say("  y rel", rel(y, y_or), "v rel", abs(v - v_or) / v_or)
        assert rel(y, y_or) < TOL and abs(v - v_or) / v_or < TOL


@pytest.mark.parametrize("C,H,W,pre", [(1, 64, 64, 0), (1, 64, 64, 6), (3, 36, 40, 2), (1, 50, 97, 1), (1, 512, 512, 1)])
def test_bf16_train_step_teacher_forced(C, H, W, pre):
    say("bf16 step", C, H, W, pre)
    clean = synth.blobs(H, W, 2, C=C)
    noisy = synth.add_gaussian(clean, 25 / 255, 12)
    r = n2f.Run(dev(noisy), bf16_cfg())
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    pairs = O.training_pairs(xs)
    for k in range(C):
        st = O.new_state(th0[k])
        for s in range(pre):
            st = O.train_step(st, C, pairs[s % 4][0], pairs[s % 4][1][k], H0)[0]
        r.set_state(k, st.theta, st.m, st.v, st.t)
        st32 = O.NetState(st.theta.astype(np.float32).astype(np.float64), st.m.astype(np.float32).astype(np.float64),
                          st.v.astype(np.float32).astype(np.float64), st.t)
        pair = pre % 4
        r.train_step(k, pair)
        g, loss = r.get_grad(k)
        _, g_or, loss_or, _ = O.train_step(st32, C, pairs[pair][0], pairs[pair][1][k], H0)
        errs = {nm: rel(a, b) for (nm, a), b in zip(split(g, C).items(), split(g_or, C).values())}
        say("  worst grad err", max(errs.values()), max(errs, key=errs.get))
        assert max(errs.values()) < TOL, errs
        assert abs(loss - loss_or) / abs(loss_or) < TOL


@pytest.mark.parametrize("splits", [1, 16])
def test_bf16_train_step_with_fewer_weight_gradient_splits(splits):
    """A 512x384 step (training images of 384 and 512 tiles) with the
    weight gradient cut into 1 or 16 pixel splits instead of 64: same bars
    against the oracle, and a different split count changes only the order
    of the sums (the step stays within the bar of the default one)."""
    say("bf16 step, splits", splits)
    C, H, W = 1, 512, 384
    clean = synth.blobs(H, W, 4)
    noisy = synth.add_gaussian(clean, 25 / 255, 14)
    r = n2f.Run(dev(noisy), n2f.default_config(precision=n2f.BF16, wgrad_splits=splits))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    pairs = O.training_pairs(xs)
    st = O.new_state(synth.init_params(C, 0)[0])
    st = O.train_step(st, C, pairs[0][0], pairs[0][1][0], H0)[0]
    r.set_state(0, st.theta, st.m, st.v, st.t)
    st32 = O.NetState(st.theta.astype(np.float32).astype(np.float64), st.m.astype(np.float32).astype(np.float64),
                      st.v.astype(np.float32).astype(np.float64), st.t)
    r.train_step(0, 1)
    g, loss = r.get_grad(0)
    _, g_or, loss_or, _ = O.train_step(st32, C, pairs[1][0], pairs[1][1][0], H0)
    errs = {nm: rel(a, b) for (nm, a), b in zip(split(g, C).items(), split(g_or, C).values())}
    say("  worst grad err", max(errs.values()), max(errs, key=errs.get))
    assert max(errs.values()) < TOL, errs
    assert abs(loss - loss_or) / abs(loss_or) < TOL


def test_bf16_deterministic_and_one_shot():
    clean = synth.blobs(48, 56, 3)
    noisy = synth.add_gaussian(clean, 25 / 255, 13)
    cfg = bf16_cfg(fixed_epochs=3)
    a, sa = n2f.denoise(dev(noisy), cfg)
    b, sb = n2f.denoise(dev(noisy), cfg)
    assert sa == sb == n2f.OK and torch.equal(a, b)


@pytest.mark.timeout(900)
def test_bf16_mean_psnr_matches_fp32():
    """Mean final PSNR over 100 initial-weight seeds (256x256 blobs scene,
    sigma 25/255, full early-stopping runs): BF16 within 0.1 dB of FP32 on
    the point estimate; the standard error of the difference (about 0.05 dB
    at the measured per-run spread) is printed beside it.  A single run's
    PSNR moves by a few tenths of a dB with the initial weights and with
    rounding noise (the stopping epoch shifts), for either precision, so
    single runs are not compared."""
    n = 100
    clean, noisy = synth.single_512(25, 2, size=256)
    x = dev(noisy)
    res, eps = {}, {}
    for name, prec in [("fp32", n2f.FP32), ("bf16", n2f.BF16)]:
        ps, ep = [], []
        for seed in range(n):
            r = n2f.Run(x, n2f.default_config(precision=prec, init_seed=seed))
            done, status = r.run_epochs(0, 2000)
            assert done and status == n2f.OK
            ps.append(synth.psnr(r.result().cpu().numpy(), clean))
            ep.append(r.progress(0)[0])
        res[name], eps[name] = np.array(ps), np.array(ep)
        say(name, "mean %.3f std %.3f, epochs %.1f" % (res[name].mean(), res[name].std(ddof=1), eps[name].mean()))
    diff = res["bf16"].mean() - res["fp32"].mean()
    se = np.sqrt(res["bf16"].var(ddof=1) / n + res["fp32"].var(ddof=1) / n)
    say("bf16 - fp32 %+.3f dB over %d seeds, standard error %.3f" % (diff, n, se))
    assert abs(diff) <= 0.1
    assert res["bf16"].min() > synth.psnr(noisy, clean) + 10.0
