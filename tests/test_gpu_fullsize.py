"""Full-size paths against the CPU FP64 oracle, at sizes where every tile
group of the BF16 convolution grid (at most 256 blocks x 2 groups of 16x16
tiles) runs several tiles: the head sums of the fused training head and the
validation squared-error sums carried across tiles, the next-tile prefetch,
and weight-gradient splits of many tiles each.  768x768 gives training images
of 768x384 and 384x768 (1152 tiles each); 1040x520 gives 1040x260 and 520x520
with ragged last tile columns and rows (260 = 16*16 + 4, 520 = 32*16 + 8).

Bars: teacher-forced training step within norm-wise relative error 1e-5
(FP32) or 2e-2 (BF16) per parameter tensor, loss and Adam moments compared;
the validation output element-wise: |y - y_oracle| <= 2^-7 max|y_oracle|
(BF16) or 1e-5 max|y_oracle| (FP32) at every pixel, tile borders included.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import n2f_oracle as O
from paper_2108_10209_amd import n2f, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H0 = O.Hyper()
TOL = {n2f.FP32: 1e-5, n2f.BF16: 2e-2}
ELEM = {n2f.FP32: 1e-5, n2f.BF16: 2.0 ** -7}
NAME = {n2f.FP32: "fp32", n2f.BF16: "bf16"}


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


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [n2f.FP32, n2f.BF16])
@pytest.mark.parametrize("H,W", [(768, 768), (1040, 520)])
def test_full_size_steps_and_validation(prec, H, W):
    """From the initial weights: a step on pair 0 (the up pair), then from
    the oracle's state after it a step on pair 2 (the left pair, the other
    training shape); then the validation forward of the oracle's state after
    both, compared pixel by pixel."""
    say(f"full-size {NAME[prec]} {H}x{W}")
    clean = synth.blobs(H, W, 4)
    noisy = synth.add_gaussian(clean, 25 / 255, 14)
    r = n2f.Run(dev(noisy), n2f.default_config(precision=prec))
    xs = r.image(4).cpu().numpy().astype(np.float64)
    pairs = O.training_pairs(xs)
    st = O.new_state(synth.init_params(1, 0)[0])
    tol = TOL[prec]
    for pair in (0, 2):
        r.set_state(0, st.theta, st.m, st.v, st.t)
        st32 = O.NetState(f32(st.theta), f32(st.m), f32(st.v), st.t)
        r.train_step(0, pair)
        g, loss = r.get_grad(0)
        inp, tgt = pairs[pair]
        st_or, g_or, loss_or, _ = O.train_step(st32, 1, inp, tgt[0], H0)
        errs = {nm: rel(a, b) for (nm, a), b in zip(split(g, 1).items(), split(g_or, 1).values())}
        worst = max(errs, key=errs.get)
        th, m, v, t = r.get_state(0)
        say(f"  pair {pair} {inp.shape[1]}x{inp.shape[2]}: worst grad err {errs[worst]:.2e} ({worst}), "
            f"loss err {abs(loss - loss_or) / abs(loss_or):.2e}, m err {rel(m, st_or.m):.2e}")
        assert errs[worst] < tol, errs
        assert abs(loss - loss_or) / abs(loss_or) < tol
        assert t == st.t + 1
        assert rel(m, st_or.m) < tol and rel(v, st_or.v) < 2 * tol
        st = st_or
    # validation of the state after both steps, every pixel
    r.set_state(0, st.theta, st.m, st.v, st.t)
    v, _, _ = r.validate(0)
    y = r.image(5).cpu().numpy().astype(np.float64).reshape(H, W)
    y_or, v_or = O.validate(f32(st.theta), 1, xs, 0, H0)
    y_or = np.asarray(y_or).reshape(H, W)
    err = np.abs(y - y_or)
    bound = ELEM[prec] * np.abs(y_or).max()
    # pixels on 16x16 tile borders, where the halo and the fused epilogues meet
    border = np.zeros_like(err, bool)
    border[::16, :] = border[15::16, :] = border[:, ::16] = border[:, 15::16] = True
    say(f"  validation: max |y - y_or| {err.max():.3e} (border {err[border].max():.3e}), bound {bound:.3e}, "
        f"score err {abs(v - v_or) / v_or:.2e}, output range [{y_or.min():.3f}, {y_or.max():.3f}]")
    assert err.max() <= bound
    assert abs(v - v_or) / v_or < tol
