"""Pins of the oracle's network, loss, gradients and optimiser against brute
force, closed forms and independent library routines (scipy, PyTorch CPU in
FP64)."""
import math

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import synth

torch.set_default_dtype(torch.float64)


def _direct_conv(a, W, b):
    """Six nested loops over the definition of a zero-padded 3x3 conv."""
    Cin, H, Wd = a.shape
    Cout = W.shape[0]
    out = np.zeros((Cout, H, Wd))
    for o in range(Cout):
        for i in range(H):
            for j in range(Wd):
                s = b[o]
                for c in range(Cin):
                    for u in range(3):
                        for v in range(3):
                            y, x = i + u - 1, j + v - 1
                            if 0 <= y < H and 0 <= x < Wd:
                                s += W[o, c, u, v] * a[c, y, x]
                out[o, i, j] = s
    return out


@pytest.mark.parametrize("Cin,Cout,H,W", [(1, 2, 5, 4), (3, 4, 4, 6), (2, 3, 1, 1), (2, 2, 2, 7)])
def test_conv_brute_force(Cin, Cout, H, W):
    rng = np.random.default_rng(Cin * 10 + H)
    a = rng.standard_normal((Cin, H, W))
    Wt = rng.standard_normal((Cout, Cin, 3, 3))
    b = rng.standard_normal(Cout)
    np.testing.assert_allclose(O.conv3x3(a, Wt, b), _direct_conv(a, Wt, b), rtol=1e-13, atol=1e-13)


def test_conv_single_channel_is_correlate2d():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(4)
    a = rng.standard_normal((1, 9, 12))
    k = rng.standard_normal((3, 3))
    out = O.conv3x3(a, k[None, None], np.zeros(1))[0]
    ref = correlate2d(a[0], k, mode="same", boundary="fill", fillvalue=0)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_conv_impulse_response():
    """A unit impulse returns the taps, mirrored about the centre."""
    a = np.zeros((1, 7, 7))
    a[0, 3, 3] = 1.0
    k = np.arange(9, dtype=np.float64).reshape(3, 3) + 1
    out = O.conv3x3(a, k[None, None], np.zeros(1))[0]
    np.testing.assert_array_equal(out[2:5, 2:5], k[::-1, ::-1])
    assert np.count_nonzero(out) == 9


def test_conv_matches_torch():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((5, 11, 8))
    Wt = rng.standard_normal((6, 5, 3, 3))
    b = rng.standard_normal(6)
    ref = torch.nn.functional.conv2d(torch.tensor(a)[None], torch.tensor(Wt), torch.tensor(b), padding=1)[0]
    np.testing.assert_allclose(O.conv3x3(a, Wt, b), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_conv_backward_matches_torch_autograd():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((4, 7, 9))
    Wt = rng.standard_normal((3, 4, 3, 3))
    d = rng.standard_normal((3, 7, 9))
    at = torch.tensor(a, requires_grad=True)
    wt = torch.tensor(Wt, requires_grad=True)
    bt = torch.zeros(3, requires_grad=True)
    out = torch.nn.functional.conv2d(at[None], wt, bt, padding=1)[0]
    (out * torch.tensor(d)).sum().backward()
    dW, db, da = O.conv3x3_backward(a, Wt, d)
    np.testing.assert_allclose(dW, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(da, at.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_sigmoid_and_bce_against_torch():
    rng = np.random.default_rng(7)
    z = rng.standard_normal((13, 9)) * 6
    z[0, 0], z[0, 1] = 40.0, -40.0
    t = rng.uniform(-0.1, 1.1, (13, 9))     # unclipped targets may leave [0, 1]
    np.testing.assert_allclose(O.sigmoid(z), torch.sigmoid(torch.tensor(z)).numpy(), rtol=1e-15, atol=0)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(z), torch.tensor(t)).item()
    assert abs(O.bce_loss(z, t) - ref) < 1e-13
    # away from saturation it is the probability-form BCE as well
    zz, tt = z[1:5], np.clip(t[1:5], 0, 1)
    p = torch.sigmoid(torch.tensor(zz))
    ref2 = torch.nn.functional.binary_cross_entropy(p, torch.tensor(tt)).item()
    assert abs(O.bce_loss(zz, tt) - ref2) < 1e-10


def test_bce_grad_finite_difference():
    rng = np.random.default_rng(8)
    z = rng.standard_normal((5, 6))
    t = rng.uniform(0, 1, (5, 6))
    g = O.bce_grad(z, t)
    h = 1e-6
    for idx in [(0, 0), (2, 3), (4, 5)]:
        zp, zm = z.copy(), z.copy()
        zp[idx] += h
        zm[idx] -= h
        fd = (O.bce_loss(zp, t) - O.bce_loss(zm, t)) / (2 * h)
        assert abs(fd - g[idx]) < 1e-9


def _tiny(C, width, n_layers, H, W, seed):
    rng = np.random.default_rng(seed)
    spec = O.param_spec(C, width, n_layers)
    theta = np.concatenate([rng.uniform(-0.6, 0.6, int(np.prod(s))) for _, s in spec])
    x = rng.uniform(0, 1, (C, H, W))
    t = rng.uniform(0, 1, (H, W))
    return theta, x, t


@pytest.mark.parametrize("C,width,n_layers", [(1, 4, 3), (1, 4, 8), (3, 3, 2), (1, (2, 3, 4, 5), 4),
                                              (2, (2, 2, 3, 3, 4, 4, 5, 5), 8)])
def test_gradients_central_differences(C, width, n_layers):
    """Every parameter tensor's gradient against central differences."""
    h = O.Hyper(width=width, n_layers=n_layers)
    theta, x, t = _tiny(C, width, n_layers, 6, 8, 10 + n_layers)
    _, g, _ = O.gradients(theta, C, x, t, h)

    def loss(th):
        params = O.unflatten(th, C, width, n_layers)
        _, z, _ = O.forward(params, x, n_layers)
        return O.bce_loss(z, t)

    rng = np.random.default_rng(0)
    eps = 1e-6
    o = 0
    checked = 0
    for name, shape in O.param_spec(C, width, n_layers):
        n = int(np.prod(shape))
        for i in rng.choice(n, size=min(n, 6), replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[o + i] += eps
            tm[o + i] -= eps
            fd = (loss(tp) - loss(tm)) / (2 * eps)
            assert abs(fd - g[o + i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (name, i, fd, g[o + i])
            checked += 1
        o += n
    assert checked > 0


def _torch_net(C, width, n_layers):
    ws = [width] * n_layers if isinstance(width, int) else list(width)
    layers = []
    cin = C
    for wl in ws:
        layers += [torch.nn.Conv2d(cin, wl, 3, padding=1), torch.nn.ReLU()]
        cin = wl
    layers.append(torch.nn.Conv2d(cin, 1, 1))
    return torch.nn.Sequential(*layers)


def _load(net, theta, C, width, n_layers):
    params = O.unflatten(theta, C, width, n_layers)
    convs = [m for m in net if isinstance(m, torch.nn.Conv2d)]
    with torch.no_grad():
        for l, m in enumerate(convs, start=1):
            m.weight.copy_(torch.tensor(params[f"W{l}"]))
            m.bias.copy_(torch.tensor(params[f"b{l}"]))


def _read(net):
    return np.concatenate([np.concatenate([m.weight.detach().numpy().ravel(), m.bias.detach().numpy().ravel()])
                           for m in net if isinstance(m, torch.nn.Conv2d)])


@pytest.mark.parametrize("C", [1, 3])
def test_train_steps_match_torch_adam(C):
    """Four train steps (one per pair, table order) against a PyTorch CPU
    FP64 model trained with BCE-with-logits and torch.optim.Adam(lr=1e-3)."""
    width, n_layers = 8, 8
    h = O.Hyper(width=width, n_layers=n_layers)
    rng = np.random.default_rng(20 + C)
    spec = O.param_spec(C, width, n_layers)
    theta = np.concatenate([rng.uniform(-0.3, 0.3, int(np.prod(s))) for _, s in spec])
    x = rng.uniform(0, 1, (C, 10, 12))
    xs, _, _ = O.standardize(x)
    pairs = O.training_pairs(xs)
    k = C - 1
    net = _torch_net(C, width, n_layers)
    _load(net, theta, C, width, n_layers)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    st = O.new_state(theta)
    for _ in range(2):
        for inp, tgt in pairs:
            st, g, loss, y = O.train_step(st, C, inp, tgt[k], h)
            opt.zero_grad()
            z = net(torch.tensor(inp)[None])[0, 0]
            lt = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(tgt[k]))
            lt.backward()
            opt.step()
            assert abs(lt.item() - loss) < 1e-12
    np.testing.assert_allclose(st.theta, _read(net), rtol=0, atol=1e-12)
    assert st.t == 8


@pytest.mark.parametrize("C", [1, 3])
def test_literal_width_train_steps_match_torch_adam(C):
    """The Methods' own widths (32, 32, 64, 64, 128, 128, 256, 256): four
    train steps against a PyTorch CPU FP64 model of those layer shapes
    trained with BCE-with-logits and torch.optim.Adam(lr=1e-3), from the
    library's initial weights for that net."""
    widths, n_layers = O.LITERAL_WIDTHS, 8
    h = O.Hyper(width=widths, n_layers=n_layers)
    theta = synth.init_params(C, 7, widths)[C - 1].astype(np.float64)
    x = np.random.default_rng(30 + C).uniform(0, 1, (C, 12, 10))
    xs, _, _ = O.standardize(x)
    pairs = O.training_pairs(xs)
    k = C - 1
    net = _torch_net(C, widths, n_layers)
    _load(net, theta, C, widths, n_layers)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    st = O.new_state(theta)
    for inp, tgt in pairs:
        st, g, loss, y = O.train_step(st, C, inp, tgt[k], h)
        opt.zero_grad()
        z = net(torch.tensor(inp)[None])[0, 0]
        lt = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(tgt[k]))
        lt.backward()
        opt.step()
        assert abs(lt.item() - loss) < 1e-12
    np.testing.assert_allclose(st.theta, _read(net), rtol=0, atol=1e-12)
    # validation output of the trained net equals the torch model's sigmoid
    yv, v = O.validate(st.theta, C, xs, k, h)
    with torch.no_grad():
        yt = torch.sigmoid(net(torch.tensor(xs)[None])[0, 0]).numpy()
    np.testing.assert_allclose(yv, yt, rtol=0, atol=1e-12)
    assert abs(v - float(np.mean((yt - xs[k]) ** 2))) < 1e-14


def test_literal_width_parameter_count():
    """Closed form: sum over layers of w_l (9 w_{l-1} + 1), w_0 = C, plus the
    head's w_8 + 1."""
    for C in (1, 2, 3):
        ws = [C] + list(O.LITERAL_WIDTHS)
        closed = sum(ws[l] * (9 * ws[l - 1] + 1) for l in range(1, 9)) + ws[8] + 1
        assert sum(int(np.prod(s)) for _, s in O.param_spec(C, O.LITERAL_WIDTHS)) == closed
        assert synth.n_params(C, synth.LITERAL_WIDTHS) == closed
    assert O.LITERAL_WIDTHS == synth.LITERAL_WIDTHS


def test_forward_shapes_and_range():
    C = 1
    theta = synth.init_params(C, 0)[0]
    params = O.unflatten(theta, C)
    x = np.random.default_rng(0).uniform(0, 1, (1, 8, 10))
    acts, z, y = O.forward(params, x)
    assert len(acts) == 9 and all(a.shape[1:] == (8, 10) for a in acts)
    assert acts[1].shape[0] == 64 and z.shape == (8, 10)
    assert np.all((y > 0) & (y < 1))
    assert np.all(acts[3] >= 0)


def test_adam_first_step_closed_form():
    """First step moves each weight by lr * g / (|g| + eps)."""
    h = O.Hyper()
    g = np.array([1e-3, -2.0, 5e-9, 0.0, 7.0])
    th0 = np.zeros(5)
    th, m, v, t = O.adam_step(th0, g, np.zeros(5), np.zeros(5), 0, h)
    np.testing.assert_allclose(th, -h.lr * g / (np.abs(g) + h.eps), rtol=1e-12, atol=0)
    assert t == 1


def test_adam_constant_gradient():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step is lr * g / (|g| + eps)."""
    h = O.Hyper()
    g = np.array([0.5, -3.0, 1e-4])
    th, m, v, t = np.zeros(3), np.zeros(3), np.zeros(3), 0
    for step in range(1, 30):
        th_prev = th
        th, m, v, t = O.adam_step(th, g, m, v, t, h)
        np.testing.assert_allclose(m / (1 - h.beta1 ** t), g, rtol=1e-12)
        np.testing.assert_allclose(v / (1 - h.beta2 ** t), g * g, rtol=1e-12)
        np.testing.assert_allclose(th - th_prev, -h.lr * g / (np.abs(g) + h.eps), rtol=1e-9)


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    h = O.Hyper()
    th = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(th.copy()))
    opt = torch.optim.Adam([p], lr=1e-3)
    m, v, t = np.zeros(50), np.zeros(50), 0
    for _ in range(12):
        g = rng.standard_normal(50)
        th, m, v, t = O.adam_step(th, g, m, v, t, h)
        p.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=0, atol=1e-13)


def test_validation_mse_fp64():
    C = 1
    theta = synth.init_params(C, 3)[0]
    x = np.random.default_rng(1).uniform(0, 1, (1, 12, 10))
    y, v = O.validate(theta, C, x, 0, O.Hyper())
    assert abs(v - math.fsum(((y - x[0]) ** 2).ravel()) / y.size) < 1e-16


def _cb_pairs_by_loops(xs):
    """The four checkerboard pairs written as plain loops (0-based; the
    complementary parity class of each row/column packed in order), for the
    routing check below."""
    C, H, W = xs.shape
    ue = np.empty((C, H, W // 2)); uo = np.empty_like(ue)
    le = np.empty((C, H // 2, W)); lo_ = np.empty_like(le)
    for c in range(C):
        for i in range(H):
            for j in range(W // 2):
                ue[c, i, j] = xs[c, i, 2 * j + (i % 2)]
                uo[c, i, j] = xs[c, i, 2 * j + 1 - (i % 2)]
        for i in range(H // 2):
            for j in range(W):
                le[c, i, j] = xs[c, 2 * i + (j % 2), j]
                lo_[c, i, j] = xs[c, 2 * i + 1 - (j % 2), j]
    return [(ue, uo), (uo, ue), (le, lo_), (lo_, le)]


def test_rgb_routing_matches_torch_per_channel_nets():
    """Multi-channel images (Fig. 2a caption: RGB predicted one channel at a
    time; Methods, validation paragraph).  A PyTorch FP64 run of two fixed
    epochs with three independent networks: network k sees all three input
    channels, trains on target channel k, is validated by MSE against
    channel k of the standardised input and writes output channel k.  The
    oracle's per-network scores, its validate() for every k and its output
    channels must all agree with it; training every network on channel 0, or
    scoring against channel 0, fails here because the channels differ."""
    C, H, W, width, n_layers, E = 3, 8, 10, 6, 3, 2
    h = O.Hyper(width=width, n_layers=n_layers, fixed_epochs=E)
    rng = np.random.default_rng(77)
    spec = O.param_spec(C, width, n_layers)
    theta0 = np.stack([np.concatenate([rng.uniform(-0.4, 0.4, int(np.prod(s))) for _, s in spec])
                       for _ in range(C)])
    x = rng.uniform(0, 1, (C, H, W)) * np.array([1.0, 0.6, 0.3])[:, None, None] + np.array([0, 0.3, 0.5])[:, None,
                                                                                                        None]
    xs = (x - x.min()) / (x.max() - x.min())
    pairs = _cb_pairs_by_loops(xs)
    ref_y, ref_hist, ref_theta = [], [], []
    for k in range(C):
        net = _torch_net(C, width, n_layers)
        _load(net, theta0[k], C, width, n_layers)
        opt = torch.optim.Adam(net.parameters(), lr=1e-3)
        hist = []
        for _ in range(E):
            for inp, tgt in pairs:
                opt.zero_grad()
                z = net(torch.tensor(inp)[None])[0, 0]
                torch.nn.functional.binary_cross_entropy_with_logits(z, torch.tensor(tgt[k])).backward()
                opt.step()
            with torch.no_grad():
                y = torch.sigmoid(net(torch.tensor(xs)[None])[0, 0]).numpy()
            hist.append(float(np.mean((y - xs[k]) ** 2)))
        ref_y.append(y)
        ref_hist.append(hist)
        ref_theta.append(_read(net))
    r = O.denoise(x, theta0, h)
    for k in range(C):
        np.testing.assert_allclose(r.history[k], ref_hist[k], rtol=1e-10, atol=0)
        np.testing.assert_allclose(r.y_std[k], ref_y[k], rtol=0, atol=1e-12)
        yk, vk = O.validate(ref_theta[k], C, xs, k, h)
        np.testing.assert_allclose(yk, ref_y[k], rtol=0, atol=1e-12)
        assert abs(vk - ref_hist[k][-1]) <= 1e-12 * ref_hist[k][-1]
    # the routing is visible: networks and their scores differ per channel
    assert min(abs(ref_hist[0][-1] - ref_hist[1][-1]), abs(ref_hist[1][-1] - ref_hist[2][-1])) > 1e-4
    np.testing.assert_allclose(r.y, O.destandardize(r.y_std, x.min(), x.max()), rtol=0, atol=1e-12)
