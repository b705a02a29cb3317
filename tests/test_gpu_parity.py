"""GPU library vs the CPU FP64 oracle, through the C ABI.

Bars: downsampling and indexing bit-exact; the standardised image within one
FP32 ulp of the oracle's FP64 value; a teacher-forced training step (GPU
loaded with the oracle's state) within norm-wise relative error 1e-5 per
parameter tensor (FP32); final PSNR within 0.1 dB.
"""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth

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


def noisy_image(C, H, W, seed, sigma=25 / 255):
    clean = synth.blobs(H, W, seed, C=C)
    return clean, synth.add_gaussian(clean, sigma, seed + 100)


# ---------------------------------------------------------------------------
# data preparation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("C,H,W", [(1, 64, 64), (1, 37, 50), (3, 33, 17), (1, 2, 2), (3, 130, 96), (1, 512, 512)])
def test_prepare_bit_exact(C, H, W):
    say("prepare", C, H, W)
    rng = np.random.default_rng(H * W + C)
    x = (rng.standard_normal((C, H, W)) * 2 + 1).astype(np.float32)
    r = n2f.Run(dev(x))
    lo, hi = r.lohi()
    assert lo == float(x.min()) and hi == float(x.max())
    xs = r.image(4).cpu().numpy()
    xs_or, _, _ = O.standardize(x)
    ulp = np.abs(xs.view(np.int32).astype(np.int64) - xs_or.astype(np.float32).view(np.int32).astype(np.int64))
    assert ulp.max() <= 1
    ue, uo = O.checkerboard_up(xs.astype(np.float64))
    le, lo_ = O.checkerboard_left(xs.astype(np.float64))
    for which, ref in enumerate([ue, uo, le, lo_]):
        got = r.image(which).cpu().numpy()
        assert got.shape == ref.shape
        np.testing.assert_array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("C,H,W", [(1, 16, 16), (2, 9, 14), (3, 64, 62)])
def test_index_image_downsample(C, H, W):
    """On the index image every downsample pixel names its source pixel."""
    say("index", C, H, W)
    x = synth.index_image(C, H, W)
    r = n2f.Run(dev(x))
    n = C * H * W - 1
    ue, uo = O.checkerboard_up(x.astype(np.float64))
    le, lo = O.checkerboard_left(x.astype(np.float64))
    for which, ref in enumerate([ue, uo, le, lo]):
        got = np.rint(r.image(which).cpu().numpy().astype(np.float64) * n)
        np.testing.assert_array_equal(got, ref)


def test_constant_and_nonfinite_inputs():
    x = np.full((1, 12, 10), 0.3, np.float32)
    y, st = n2f.denoise(dev(x))
    assert st == n2f.WCONSTANT and torch.equal(y.cpu(), torch.from_numpy(x))
    x[0, 3, 4] = np.nan
    with pytest.raises(n2f.N2FError) as e:
        n2f.Run(dev(x))
    assert e.value.code == n2f.EINVAL


# ---------------------------------------------------------------------------
# forward pass / validation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("C,H,W", [(1, 64, 64), (1, 45, 70), (3, 40, 33), (1, 17, 130)])
def test_validation_matches_oracle(C, H, W):
    say("validate", C, H, W)
    _, noisy = noisy_image(C, H, W, 1)
    r = n2f.Run(dev(noisy))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    for k in range(C):
        v, imp, done = r.validate(k)
        y = r.image(5 + k).cpu().numpy()
        y_or, v_or = O.validate(th0[k], C, xs, k, H0)
        assert rel(y, y_or) < 1e-5
        assert abs(v - v_or) / v_or < 1e-5
        assert imp and not done
        assert r.progress(k)[:3] == (1, 1, 0)


# ---------------------------------------------------------------------------
# teacher-forced training steps
# ---------------------------------------------------------------------------
def _oracle_state(C, k, xs, steps, th0):
    st = O.new_state(th0[k])
    pairs = O.training_pairs(xs)
    for s in range(steps):
        inp, tgt = pairs[s % 4]
        st, _, _, _ = O.train_step(st, C, inp, tgt[k], H0)
    return st, pairs


def _check_step(r, C, k, st, pairs, pair, tol=1e-5):
    r.set_state(k, st.theta, st.m, st.v, st.t)
    # what the GPU actually starts from (FP32-rounded oracle state)
    th32 = st.theta.astype(np.float32).astype(np.float64)
    st32 = O.NetState(th32, st.m.astype(np.float32).astype(np.float64),
                      st.v.astype(np.float32).astype(np.float64), st.t)
    r.train_step(k, pair)
    g, loss = r.get_grad(k)
    inp, tgt = pairs[pair]
    st_or, g_or, loss_or, _ = O.train_step(st32, C, inp, tgt[k], H0)
    gg, go = split(g, C), split(g_or, C)
    errs = {name: rel(gg[name], go[name]) for name in gg}
    assert max(errs.values()) < tol, errs
    assert abs(loss - loss_or) / abs(loss_or) < 1e-6
    th, m, v, t = r.get_state(k)
    assert t == st.t + 1
    assert rel(m, st_or.m) < tol and rel(v, st_or.v) < 2 * tol
    return errs, th, st_or


@pytest.mark.parametrize("C,H,W,pre", [(1, 64, 64, 0), (1, 64, 64, 5), (1, 50, 38, 2), (3, 40, 36, 3),
                                       (1, 33, 97, 1)])
def test_train_step_teacher_forced(C, H, W, pre):
    say("train step", C, H, W, pre)
    _, noisy = noisy_image(C, H, W, 2)
    r = n2f.Run(dev(noisy))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    for k in range(C):
        st, pairs = _oracle_state(C, k, xs, pre, th0)
        _check_step(r, C, k, st, pairs, pre % 4)


def test_adam_with_injected_gradient():
    C = 1
    _, noisy = noisy_image(C, 32, 32, 3)
    r = n2f.Run(dev(noisy))
    rng = np.random.default_rng(0)
    npar = synth.n_params(C)
    th = rng.standard_normal(npar).astype(np.float32) * 0.05
    m = rng.standard_normal(npar).astype(np.float32) * 1e-3
    v = np.abs(rng.standard_normal(npar)).astype(np.float32) * 1e-6
    g = rng.standard_normal(npar).astype(np.float32) * 1e-3
    r.set_state(0, th, m, v, 7)
    r.debug_adam(0, g)
    th2, m2, v2, t2 = r.get_state(0)
    th_or, m_or, v_or, t_or = O.adam_step(th.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                          v.astype(np.float64), 7, H0)
    assert t2 == t_or == 8
    assert rel(th2 - th, th_or - th) < 1e-5
    assert rel(m2, m_or) < 1e-6 and rel(v2, v_or) < 1e-6


def test_full_size_step_and_validation_512():
    """512x512 (the benchmark's image size): one teacher-forced step from a
    state 4 steps in, and the full-image validation output afterwards."""
    say("512 step")
    C = 1
    _, noisy = synth.single_512(25, 2)
    r = n2f.Run(dev(noisy))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    th0 = synth.init_params(C, 0)
    st, pairs = _oracle_state(C, 0, xs, 4, th0)
    errs, th, st_or = _check_step(r, C, 0, st, pairs, 0)
    say("512 grad errs", max(errs.values()))
    r.set_state(0, st_or.theta, st_or.m, st_or.v, st_or.t)
    v, imp, done = r.validate(0)
    y = r.image(5).cpu().numpy()
    y_or, v_or = O.validate(st_or.theta.astype(np.float32).astype(np.float64), C, xs, 0, H0)
    assert rel(y, y_or) < 1e-5 and abs(v - v_or) / v_or < 1e-5


# ---------------------------------------------------------------------------
# whole loop
# ---------------------------------------------------------------------------
def test_small_64_fixed_8_epochs():
    """64x64, sigma 25/255, 8 fixed epochs (32 steps): every step teacher-
    forced within 1e-5; the free-running validation scores within 1e-3 of
    the oracle's; the one-shot entry point equals the step-wise run."""
    say("64x64 8 epochs")
    clean, noisy = synth.small_64(0)
    th0 = synth.init_params(1, 0)
    cfg = n2f.default_config(fixed_epochs=8)
    r = n2f.Run(dev(noisy), cfg)
    xs = r.image(4).cpu().numpy().astype(np.float64)
    st = O.new_state(th0[0])
    pairs = O.training_pairs(xs)
    worst = 0.0
    for e in range(8):
        for p in range(4):
            errs, _, st_next = _check_step(r, 1, 0, st, pairs, p)
            worst = max(worst, max(errs.values()))
            st = O.train_step(st, 1, pairs[p][0], pairs[p][1][0], H0)[0]
    say("worst teacher-forced grad err", worst)
    # free run on the GPU from the same initial weights
    r2 = n2f.Run(dev(noisy), cfg)
    done, status = r2.run_epochs(0, 8)
    assert done and status == n2f.OK
    y = r2.result().cpu().numpy()
    ref = O.denoise(noisy, th0, O.Hyper(fixed_epochs=8))
    p_gpu, p_or = synth.psnr(y, clean), synth.psnr(ref.y, clean)
    # reported only: this one seed's free-running PSNR flips between the
    # oracle's value and a few tenths of a dB off with the rounding of a single
    # step (8 epochs of a fresh net are chaotic); the PSNR gate is the paired
    # mean over 64 seeds in test_fixed_8_epochs_psnr_matches_oracle_over_seeds
    say("psnr gpu", p_gpu, "oracle", p_or, "diff %+.4f dB (report only)" % (p_gpu - p_or),
        "noisy", synth.psnr(noisy, clean))
    hist = r2.history(0)
    assert len(hist) == 8
    np.testing.assert_allclose(hist, ref.history[0], rtol=1e-3)
    # one-shot entry point gives the same bits as the step-wise run
    y1, st1 = n2f.denoise(dev(noisy), cfg)
    assert st1 == n2f.OK and torch.equal(y1.cpu(), torch.from_numpy(y))


def test_stopping_rule_and_output_average():
    """Device-side stopping rule (patience 10), driven step by step with every
    epoch's output read back: the device improves and stops exactly where the
    oracle's rule, fed the GPU's own scores, does; the result is the mean of
    the outputs after the best epoch; the queued-epochs path gives the same
    bits as the step-wise one."""
    say("early stop 40x48")
    clean, noisy = noisy_image(1, 40, 48, 5)
    cfg = n2f.default_config(patience=10, max_epochs=300)
    r = n2f.Run(dev(noisy), cfg)
    lo, hi = r.lohi()
    es = O.EarlyStop(10)
    for e in range(300):
        for p in range(4):
            r.train_step(0, p)
        v, imp, done = r.validate(0)
        y = r.image(5).cpu().numpy().astype(np.float64)
        imp_or, done_or = es.update(y, v)
        assert (imp, done) == (imp_or, done_or), e
        if done:
            break
    assert done
    ep, be, ns, best = r.progress(0)
    assert (ep, be, ns) == (es.epoch, es.best_epoch, 10) and best == es.best
    np.testing.assert_array_equal(r.history(0), np.array(es.history))
    out = r.result().cpu().numpy()
    assert rel(out[0], lo + (hi - lo) * es.output()) < 1e-6
    r2 = n2f.Run(dev(noisy), cfg)
    done2, status = r2.run_epochs(0, 300)
    assert done2 and status == n2f.OK
    assert torch.equal(r2.result().cpu(), torch.from_numpy(out))
    say("epochs", ep, "best", be, "psnr", synth.psnr(out, clean), "noisy", synth.psnr(noisy, clean))
    assert synth.psnr(out, clean) > synth.psnr(noisy, clean) + 3.0


def test_cap_reports_warning():
    _, noisy = noisy_image(1, 20, 24, 8)
    cfg = n2f.default_config(patience=50, max_epochs=3)
    r = n2f.Run(dev(noisy), cfg)
    done, status = r.run_epochs(0, 10)
    assert done and status == n2f.WCAPPED and r.progress(0)[0] == 3
    with pytest.raises(n2f.N2FError) as e:
        r.train_step(0, 0)
    assert e.value.code == n2f.ESTATE


def test_rgb_fixed_epochs_matches_oracle():
    say("rgb")
    clean, noisy = noisy_image(3, 24, 20, 6)
    th0 = synth.init_params(3, 0)
    cfg = n2f.default_config(fixed_epochs=2)
    y, st = n2f.denoise(dev(noisy), cfg)
    ref = O.denoise(noisy, th0, O.Hyper(fixed_epochs=2))
    for k in range(3):
        assert rel(y[k].cpu().numpy(), ref.y[k]) < 1e-4


def test_deterministic():
    _, noisy = noisy_image(1, 70, 66, 7)
    cfg = n2f.default_config(fixed_epochs=3)
    a, _ = n2f.denoise(dev(noisy), cfg)
    b, _ = n2f.denoise(dev(noisy), cfg)
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_graph_replay_equals_direct_launches(prec):
    """Epochs replayed from one recorded HIP graph (host polling between
    replays) give the same bits as epochs launched kernel by kernel, with
    a fixed epoch count and with the stopping rule firing mid-batch."""
    _, noisy = noisy_image(1, 52, 44, 9)
    for kw in [dict(fixed_epochs=5), dict(patience=5, max_epochs=80)]:
        outs = []
        for g in (1, 0):
            r = n2f.Run(dev(noisy), n2f.default_config(precision=prec, use_graph=g, **kw))
            done, status = r.run_epochs(0, 200)
            assert done and status == n2f.OK
            outs.append((r.result().cpu(), r.history(0), r.progress(0)))
        assert torch.equal(outs[0][0], outs[1][0])
        np.testing.assert_array_equal(outs[0][1], outs[1][1])
        assert outs[0][2] == outs[1][2]


def test_free_running_steps_track_oracle():
    """Eight steps with the state kept on the device (no teacher forcing):
    the accumulated parameter change stays within 1e-4 (norm-wise) of the
    oracle's.  This guards the step counter, Adam's constants (1 - beta2
    must be exact to FP32) and the weight repacking between steps."""
    _, noisy = synth.small_64(0)
    th0 = synth.init_params(1, 0)[0]
    r = n2f.Run(dev(noisy), n2f.default_config(fixed_epochs=8))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    pairs = O.training_pairs(xs)
    st = O.new_state(th0)
    for step in range(8):
        r.train_step(0, step % 4)
        st = O.train_step(st, 1, pairs[step % 4][0], pairs[step % 4][1][0], H0)[0]
    th, m, v, t = r.get_state(0)
    say("free-run dtheta err", rel(th - th0, st.theta - th0), "v err", rel(v, st.v))
    assert t == 8
    assert rel(th - th0, st.theta - th0) < 1e-4
    assert rel(v, st.v) < 1e-4


SEED_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_psnr_64_sigma25_seeds.json")
FIXED8_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_psnr_64_sigma25_fixed8_seeds.json")


@pytest.mark.timeout(600)
@pytest.mark.skipif(not os.path.exists(SEED_GOLDEN), reason="oracle seed golden not generated")
@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_mean_psnr_matches_oracle_over_seeds(prec):
    """Whole loop with early stopping (64x64, sigma 25/255): the mean final
    PSNR over the oracle's stored initial-weight seeds is within 0.1 dB of
    the oracle's mean.  A single run's PSNR moves by a few tenths of a dB
    with rounding noise (the stopping epoch shifts), so means over many
    seeds are compared; the gate is on the point estimate, and the standard
    error of the difference is printed beside it."""
    gold = json.load(open(SEED_GOLDEN))
    clean, noisy = synth.small_64(0)
    x = dev(noisy)
    ps, eps = [], []
    for run in gold["runs"]:
        r = n2f.Run(x, n2f.default_config(precision=prec, init_seed=run["seed"]))
        done, status = r.run_epochs(0, 2000)
        assert done and status == n2f.OK
        ps.append(synth.psnr(r.result().cpu().numpy(), clean))
        eps.append(r.progress(0)[0])
    ps = np.array(ps)
    po = np.array([run["psnr"] for run in gold["runs"]])
    n = len(ps)
    se = np.sqrt(ps.var(ddof=1) / n + po.var(ddof=1) / n)
    diff = ps.mean() - po.mean()
    say("%s over %d seeds: gpu mean %.3f std %.3f | oracle mean %.3f std %.3f | diff %+.3f dB, se %.3f | "
        "epochs %.1f vs %.1f" % ("bf16" if prec == n2f.BF16 else "fp32", n, ps.mean(), ps.std(ddof=1), po.mean(),
                                 po.std(ddof=1), diff, se, np.mean(eps),
                                 np.mean([run["epochs"] for run in gold["runs"]])))
    assert n >= 100   # enough seeds that the standard error is about 0.05 dB
    assert abs(diff) <= 0.1
    assert ps.min() > gold["noisy_psnr"] + 5.0


@pytest.mark.skipif(not os.path.exists(FIXED8_GOLDEN), reason="oracle fixed-epoch seed golden not generated")
@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
def test_fixed_8_epochs_psnr_matches_oracle_over_seeds(prec):
    """The 64x64 configuration (8 fixed epochs, output = the last validation
    output) from every stored initial-weight seed: the mean of the per-seed
    PSNR differences GPU - oracle is within 0.1 dB.  The runs start from the
    same weights and take the same 32 steps, so the differences are paired;
    their standard error is printed beside the point estimate."""
    gold = json.load(open(FIXED8_GOLDEN))
    clean, noisy = synth.small_64(0)
    x = dev(noisy)
    d = []
    for run in gold["runs"]:
        r = n2f.Run(x, n2f.default_config(precision=prec, init_seed=run["seed"], fixed_epochs=8))
        done, status = r.run_epochs(0, 8)
        assert done and status == n2f.OK
        d.append(synth.psnr(r.result().cpu().numpy(), clean) - run["psnr"])
    d = np.array(d)
    se = d.std(ddof=1) / np.sqrt(len(d))
    say("%s 8 fixed epochs over %d seeds: mean diff %+.4f dB, se %.4f, median |diff| %.4f, max |diff| %.3f" %
        ("bf16" if prec == n2f.BF16 else "fp32", len(d), d.mean(), se, np.median(np.abs(d)), np.abs(d).max()))
    assert abs(d.mean()) <= 0.1


GOLD_256 = os.path.join(os.path.dirname(__file__), "golden", "oracle_psnr_256_sigma25.json")


@pytest.mark.skipif(not os.path.exists(GOLD_256), reason="oracle 256 golden not generated")
def test_single_run_256_report():
    """One full early-stopping run at 256x256 (sigma 25/255, seed 0) beside
    the oracle's run on the same inputs, reported only: single runs scatter
    by about 0.4 dB (standard deviation over seeds), so one run cannot
    resolve 0.1 dB; the seed-mean tests above are the PSNR gates.  Checked:
    the run finishes and denoises (output well above the noisy PSNR)."""
    gold = json.load(open(GOLD_256))
    clean, noisy = synth.single_512(25, 2, size=256)
    r = n2f.Run(dev(noisy), n2f.default_config())
    done, status = r.run_epochs(0, 2000)
    p = synth.psnr(r.result().cpu().numpy(), clean)
    say("256 single run: gpu %.3f dB (epochs, best) %s | oracle %.3f dB (%d, %d) | diff %+.3f dB (report only)" %
        (p, r.progress(0)[:2], gold["psnr"], gold["epochs"], gold["best_epoch"], p - gold["psnr"]))
    assert done and status == n2f.OK
    assert p > synth.psnr(noisy, clean) + 5.0
