"""The tie-aware FP32 check (`fp32_ties`) on the CPU: with no decision
reversed it is the oracle's gradient; an independent FP32 evaluation (PyTorch
CPU convolutions in float32) of a state with a tied seventh-layer unit
misses the FP64 gradient by 2e-4 and lands within 1e-6 of the reversed
decision; a gradient with a decision reversed far from its tie is refused;
the fixed-epoch run it replays is the oracle's own run."""
import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import synth
import fp32_ties as T

LIT = O.LITERAL_WIDTHS


def image(C, H, W, seed):
    return synth.add_gaussian(synth.blobs(H, W, seed, C=C), 25 / 255, seed + 100)


def state_after(C, H, W, seed, pre, k, width=LIT):
    h = O.Hyper(width=width)
    xs, _, _ = O.standardize(image(C, H, W, seed))
    pairs = O.training_pairs(xs)
    st = O.new_state(synth.init_params(C, 0, width)[k])
    for s in range(pre):
        st = O.train_step(st, C, pairs[s % 4][0], pairs[s % 4][1][k], h)[0]
    theta = np.asarray(st.theta, np.float32).astype(np.float64)
    return theta, pairs[pre % 4]


def torch_fp32_gradient(theta, C, inp, tgt, width):
    prm = O.unflatten(theta, C, width)
    ws = O.layer_widths(width)
    p = {n: torch.tensor(v, dtype=torch.float32, requires_grad=True) for n, v in prm.items()}
    a = torch.tensor(inp, dtype=torch.float32)[None]
    for l in range(1, len(ws) + 1):
        a = torch.relu(torch.nn.functional.conv2d(a, p[f"W{l}"], p[f"b{l}"], padding=1))
    L = len(ws) + 1
    z = torch.nn.functional.conv2d(a, p[f"W{L}"], p[f"b{L}"])[0, 0]
    torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(tgt, dtype=torch.float32)).backward()
    g = {n: t.grad.double().numpy() for n, t in p.items()}
    return O.flatten(g, C, width)


def test_no_reversal_is_the_oracle_gradient():
    theta, (inp, tgt) = state_after(2, 14, 12, 1, 1, 1)
    _, g, _ = O.gradients(theta, 2, inp, tgt[1], O.Hyper(width=LIT))
    np.testing.assert_allclose(T.gradient_with_flips(theta, 2, inp, tgt[1], LIT, ()), g, rtol=0, atol=1e-15)


def test_torch_fp32_lands_on_the_reversed_tie():
    C, k = 3, 0
    theta, (inp, tgt) = state_after(C, 34, 30, 3, 1, k)
    units = T.tied_units(theta, C, inp, LIT)
    assert units and units[0][1] == 7 and units[0][0] < 1e-7
    g32 = torch_fp32_gradient(theta, C, inp, tgt[k], LIT)
    _, g_or, _ = O.gradients(theta, C, inp, tgt[k], O.Hyper(width=LIT))
    a, b = T.split(g32, C, LIT), T.split(g_or, C, LIT)
    assert T.rel(a["W1"], b["W1"]) > 1e-4
    ok, errs, _, flips = T.fp32_check(g32, theta, C, inp, tgt[k], LIT)
    assert ok and flips and max(errs.values()) < 1e-6, errs


def test_reversal_away_from_a_tie_is_refused():
    C, k = 1, 0
    theta, (inp, tgt) = state_after(C, 20, 18, 4, 1, k)
    prm = O.unflatten(theta, C, LIT)
    z = O.conv3x3(inp, prm["W1"], prm["b1"])
    idx = int(np.argmax(np.abs(z)))                       # the first layer's largest pre-activation
    g_bad = T.gradient_with_flips(theta, C, inp, tgt[k], LIT, ((1, idx),))
    ok, _, _, _ = T.fp32_check(g_bad, theta, C, inp, tgt[k], LIT)
    assert not ok
    ok, _, _, flips = T.fp32_check(T.gradient_with_flips(theta, C, inp, tgt[k], LIT, ()), theta, C, inp, tgt[k], LIT)
    assert ok and flips == ()


@pytest.mark.parametrize("width", [LIT, 32])
def test_fixed_run_replay_is_the_oracle_run(width):
    x = image(2, 16, 14, 11)
    th0 = synth.init_params(2, 0, width)
    h = O.Hyper(fixed_epochs=2, width=width)
    ref = O.denoise(x, th0, h)
    outs = T.fixed_run_outputs(x, th0, 1, h)
    assert outs[0][0] == "exact"
    np.testing.assert_allclose(outs[0][1], ref.y[1], rtol=0, atol=1e-13)
