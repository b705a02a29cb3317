"""Pins of the stopping rule and output averaging (Methods, validation
paragraph): stop once 100 epochs pass without improving the best validation
score and return the mean of the last 100 validation outputs."""
from collections import deque

import numpy as np
import pytest

from oracle import n2f_oracle as O


def _literal(scores, outs, patience, max_epochs=10 ** 9):
    """The rule as stated, with an explicit window of the last `patience`
    outputs and a counter of epochs since the best score."""
    best, since = np.inf, 0
    window = deque(maxlen=patience)
    for e, (v, y) in enumerate(zip(scores, outs), start=1):
        window.append(y)
        if v < best:
            best, since = v, 0
        else:
            since += 1
        if since == patience:
            return e, np.mean(np.stack(list(window)), axis=0)
        if e == max_epochs:
            return e, None
    return None, None


@pytest.mark.parametrize("kind", ["decreasing_then_flat", "ties", "late_improvement", "noisy"])
def test_running_sum_equals_window(kind):
    rng = np.random.default_rng(hash(kind) % 1000)
    patience = 100
    n = 600
    if kind == "decreasing_then_flat":
        scores = list(np.linspace(1, 0.5, 50)) + [0.6] * (n - 50)
    elif kind == "ties":
        scores = [1.0, 0.5] + [0.5] * (n - 2)        # ties never count as improvements
    elif kind == "late_improvement":
        scores = [1.0] + [1.5] * 99 + [0.9] + [2.0] * (n - 101)
    else:
        scores = list(np.abs(rng.standard_normal(n)) + np.linspace(0, 2, n))
    outs = [rng.standard_normal((3, 4)) for _ in range(n)]
    e_ref, y_ref = _literal(scores, outs, patience)
    es = O.EarlyStop(patience)
    for e, (v, y) in enumerate(zip(scores, outs), start=1):
        _, done = es.update(y, v)
        if done:
            break
    assert e == e_ref
    np.testing.assert_allclose(es.output(), y_ref, rtol=0, atol=1e-15)
    # the window is exactly the epochs after the best one
    assert e == es.best_epoch + patience


def test_ties_do_not_improve():
    es = O.EarlyStop(3)
    y = np.zeros(2)
    assert es.update(y, 1.0) == (True, False)
    assert es.update(y, 1.0) == (False, False)
    assert es.update(y, 1.0) == (False, False)
    assert es.update(y, 1.0) == (False, True)
    assert es.best_epoch == 1


def test_output_without_followers_is_best():
    es = O.EarlyStop(5)
    y1, y2 = np.full(2, 1.0), np.full(2, 2.0)
    es.update(y1, 3.0)
    es.update(y2, 2.0)
    np.testing.assert_array_equal(es.output(), y2)
    es.update(np.full(2, 4.0), 5.0)
    np.testing.assert_array_equal(es.output(), np.full(2, 4.0))


def _tiny_run(h, seed=0):
    rng = np.random.default_rng(seed)
    C = 1
    spec = O.param_spec(C, h.width, h.n_layers)
    theta0 = np.concatenate([rng.uniform(-0.5, 0.5, int(np.prod(s))) for _, s in spec])[None]
    x = rng.uniform(0, 1, (C, 6, 6)).astype(np.float32)
    return x, theta0


def test_denoise_cap_and_fixed_epochs():
    h = O.Hyper(width=4, n_layers=2, patience=3, max_epochs=4)
    x, th = _tiny_run(h)
    r = O.denoise(x, th, h)
    assert r.epochs[0] <= 4
    h2 = O.Hyper(width=4, n_layers=2, fixed_epochs=3)
    steps = []
    r2 = O.denoise(x, th, h2, trace=lambda k, e, p, st, g, l: steps.append((e, p, st.t)))
    assert r2.epochs == [3] and len(r2.history[0]) == 3
    assert [s[1] for s in steps] == [0, 1, 2, 3] * 3 and steps[-1][2] == 12
    # fixed-epoch output is the last validation output, mapped back to input units
    xs, lo, hi = O.standardize(x)
    st = O.new_state(th[0])
    pairs = O.training_pairs(xs)
    for _ in range(3):
        for inp, tgt in pairs:
            st, _, _, _ = O.train_step(st, 1, inp, tgt[0], h2)
    y, _ = O.validate(st.theta, 1, xs, 0, h2)
    np.testing.assert_allclose(r2.y[0], lo + (hi - lo) * y, rtol=0, atol=1e-14)


def test_denoise_early_stop_terminates_after_patience():
    h = O.Hyper(width=4, n_layers=2, patience=5, max_epochs=400)
    x, th = _tiny_run(h, 3)
    r = O.denoise(x, th, h)
    if not r.capped[0]:
        assert r.epochs[0] == r.best_epoch[0] + 5
        hist = r.history[0]
        assert min(hist) == hist[r.best_epoch[0] - 1]
        assert all(v >= hist[r.best_epoch[0] - 1] for v in hist[r.best_epoch[0]:])


def test_denoise_small_image_improves_psnr():
    """64x64 blobs scene, sigma 25/255, eight fixed epochs: the output is
    already closer to the clean image than the noisy input."""
    from paper_2108_10209_amd import synth
    clean, noisy = synth.small_64(0)
    r = O.denoise(noisy, synth.init_params(1, 0), O.Hyper(fixed_epochs=8))
    assert r.epochs == [8]
    assert synth.psnr(r.y, clean) > synth.psnr(noisy, clean) + 0.5
    assert all(b < a for a, b in zip(r.history[0][:3], r.history[0][1:4]))


@pytest.mark.parametrize("downsample,exact", [("quad", False), ("checkerboard", True), ("quad", True)])
def test_denoise_ablation_variants_train_on_their_pairs(downsample, exact):
    """The ablation switches of `denoise` change the training pairs only:
    the same run rebuilt step by step from `training_pairs` / `exact_pairs`
    gives the same output."""
    h = O.Hyper(width=4, n_layers=2, fixed_epochs=2)
    x, th = _tiny_run(h, 5)
    rng = np.random.default_rng(11)
    clean = x - 0.05 * rng.standard_normal(x.shape) if exact else None
    r = O.denoise(x, th, h, downsample=downsample, clean=clean)
    xs, lo, hi = O.standardize(x)
    pairs = O.exact_pairs(xs, (clean - lo) / (hi - lo), downsample) if exact else O.training_pairs(xs, downsample)
    st = O.new_state(th[0])
    for _ in range(2):
        for inp, tgt in pairs:
            st, _, _, _ = O.train_step(st, 1, inp, tgt[0], h)
    y, _ = O.validate(st.theta, 1, xs, 0, h)
    np.testing.assert_allclose(r.y[0], lo + (hi - lo) * y, rtol=0, atol=1e-14)
    plain = O.denoise(x, th, h)
    assert not np.allclose(plain.y, r.y)


def test_denoise_small_image_quad_improves_psnr():
    """The 2x2-block variant also denoises the 64x64 scene in eight epochs."""
    from paper_2108_10209_amd import synth
    clean, noisy = synth.small_64(0)
    r = O.denoise(noisy, synth.init_params(1, 0), O.Hyper(fixed_epochs=8), downsample="quad")
    assert synth.psnr(r.y, clean) > synth.psnr(noisy, clean) + 0.5
