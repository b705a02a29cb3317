"""Plain FP64 CPU reference of the Noise2Fast per-image loop.

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark run
it.  It shares no code with the GPU library: it is written from the paper
(Noise2Fast, Lequyer et al., arXiv 2108.10209) in numpy, FP64 throughout,
with images in planar (C, H, W) layout and weights in (Cout, Cin, kh, kw).

Every function names the passage it follows.  Where the paper is silent or
self-contradictory the reading taken here is stated in the function:

* standardisation is a per-image min-max map to [0, 1] with no clipping
  (Methods, "Compared Methods": images are standardised, noisy data never
  clipped; the sigmoid output and BCE target live in [0, 1]);
* the checkerboard equations are read 0-based, "odd" being the complementary
  parity class compacted (Fig. 1 caption and the "up"/"left" equations of the
  Methods section; the printed +1 form leaves the image on odd rows);
  odd image sizes drop the last row/column for the downsamples only;
* network: eight 3x3 conv+ReLU layers of width 64 with biases, zero padding,
  then a 1x1 conv and a sigmoid (Methods, network paragraph; Fig. 2a); the
  paragraph's own widths, doubling from 32 to 256 two layers at a time, are
  available as LITERAL_WIDTHS (any per-layer widths are);
  one network per output channel, each seeing all input channels (Fig. 2a
  caption on RGB);
* loss: mean binary cross-entropy over the target's pixels, in its logit form
  (Methods, training paragraph);
* optimiser: Adam, lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8 outside the root
  (Kingma and Ba, Algorithm 1), one step per pair, pairs in table order;
* validation after each epoch: MSE between the full noisy (standardised) image
  and the network output, summed in FP64;
* stop once 100 epochs pass with no strict improvement of the best validation
  score and output the mean of the last 100 validation outputs, which are the
  100 outputs after the best epoch; outputs are mapped back by the inverse of
  the standardisation;
* ablations (Methods, Ablation Study; Table 1): the 2x2-block ("Quad")
  downsamples, paired along the block diagonals in both directions (the
  pairing is not stated), and the "Exact" targets, from which the known
  signal difference between target and input is removed (the clean image
  standardised with the noisy image's extremes);
* volumes (Methods, Fluorescence Microscopy Images): every z-slice is
  denoised on its own, then the stack is max projected.

Parity pins for every function live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WIDTH = 64
N_LAYERS = 8
# The widths the Methods' network paragraph gives layer by layer: two layers
# each of 32, 64, 128 and 256 channels (the benchmark configurations use 64
# throughout; both are supported).
LITERAL_WIDTHS = (32, 32, 64, 64, 128, 128, 256, 256)


def layer_widths(width, n_layers: int = N_LAYERS):
    """Per-layer output channels: `width` is one int for every layer, or a
    sequence of n_layers ints."""
    if isinstance(width, (int, np.integer)):
        return [int(width)] * n_layers
    ws = [int(v) for v in width]
    assert len(ws) == n_layers, (ws, n_layers)
    return ws


# ---------------------------------------------------------------------------
# Parameters: canonical flat layout (W1, b1, ..., W8, b8, W9, b9), C order.
# ---------------------------------------------------------------------------
def param_spec(C: int, width=WIDTH, n_layers: int = N_LAYERS):
    """Shapes of one network's parameters (Methods, network paragraph):
    3x3 layer l maps the previous layer's channels (C for the first) to its
    own width; the 1x1 head maps the last width to one channel."""
    spec = []
    cin = C
    for l, wl in enumerate(layer_widths(width, n_layers), start=1):
        spec.append((f"W{l}", (wl, cin, 3, 3)))
        spec.append((f"b{l}", (wl,)))
        cin = wl
    spec.append((f"W{n_layers + 1}", (1, cin, 1, 1)))
    spec.append((f"b{n_layers + 1}", (1,)))
    return spec


def unflatten(theta: np.ndarray, C: int, width=WIDTH, n_layers: int = N_LAYERS) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in param_spec(C, width, n_layers):
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    assert o == theta.size, (o, theta.size)
    return out


def flatten(params: dict, C: int, width=WIDTH, n_layers: int = N_LAYERS) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], np.float64).ravel()
                           for name, _ in param_spec(C, width, n_layers)])


# ---------------------------------------------------------------------------
# Data preparation
# ---------------------------------------------------------------------------
def standardize(x: np.ndarray):
    """Per-image min-max map to [0, 1], no clipping (Methods, Compared Methods).

    Returns (x_std, lo, hi); x_std is None for a constant image, which the
    method cannot denoise and is returned unchanged.
    """
    x = np.asarray(x, dtype=np.float64)
    lo, hi = float(x.min()), float(x.max())
    if hi == lo:
        return None, lo, hi
    return (x - lo) / (hi - lo), lo, hi


def destandardize(y: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Inverse of `standardize`, mapping network outputs back to input units."""
    return lo + (hi - lo) * np.asarray(y, np.float64)


def even_extent(H: int, W: int):
    """Rows and columns used by the downsamples: odd sizes drop the last one."""
    return H - H % 2, W - W % 2


def checkerboard_up(x: np.ndarray):
    """'Up' checkerboard downsamples (Theoretical Background, Fig. 1).

    Row i keeps the pixels whose row+column parity is even (x_even) or odd
    (x_odd), packed left in column order: x_even(i, j) = x(i, 2j + i mod 2),
    x_odd(i, j) = x(i, 2j + 1 - i mod 2).  Shapes (C, H', W'/2).
    """
    C, H, W = x.shape
    Hc, Wc = even_extent(H, W)
    xe = np.empty((C, Hc, Wc // 2), dtype=x.dtype)
    xo = np.empty((C, Hc, Wc // 2), dtype=x.dtype)
    for i in range(Hc):
        p = i % 2
        xe[:, i, :] = x[:, i, p:Wc:2]
        xo[:, i, :] = x[:, i, 1 - p:Wc:2]
    return xe, xo


def checkerboard_left(x: np.ndarray):
    """'Left' checkerboard downsamples (Methods, implementation details).

    Column j keeps the pixels of even (x'_even) or odd (x'_odd) row+column
    parity, packed upward in row order: x'_even(i, j) = x(2i + j mod 2, j),
    x'_odd(i, j) = x(2i + 1 - j mod 2, j).  Shapes (C, H'/2, W').
    """
    C, H, W = x.shape
    Hc, Wc = even_extent(H, W)
    xe = np.empty((C, Hc // 2, Wc), dtype=x.dtype)
    xo = np.empty((C, Hc // 2, Wc), dtype=x.dtype)
    for j in range(Wc):
        p = j % 2
        xe[:, :, j] = x[:, p:Hc:2, j]
        xo[:, :, j] = x[:, 1 - p:Hc:2, j]
    return xe, xo


def quad_downsample(x: np.ndarray):
    """2x2-block downsamples of the ablation study (Methods, Ablation Study;
    Table 1, "Quad").

    The image is cut into 2x2 blocks; the four images hold the top-left,
    top-right, bottom-left and bottom-right pixel of every block:
    TL(i, j) = x(2i, 2j), TR(i, j) = x(2i, 2j + 1), BL(i, j) = x(2i + 1, 2j),
    BR(i, j) = x(2i + 1, 2j + 1).  Odd sizes drop the last row/column, as for
    the checkerboard.  Shapes (C, H'/2, W'/2).
    """
    C, H, W = x.shape
    Hc, Wc = even_extent(H, W)
    tl = np.empty((C, Hc // 2, Wc // 2), dtype=x.dtype)
    tr = np.empty_like(tl)
    bl = np.empty_like(tl)
    br = np.empty_like(tl)
    for i in range(Hc // 2):
        for j in range(Wc // 2):
            tl[:, i, j] = x[:, 2 * i, 2 * j]
            tr[:, i, j] = x[:, 2 * i, 2 * j + 1]
            bl[:, i, j] = x[:, 2 * i + 1, 2 * j]
            br[:, i, j] = x[:, 2 * i + 1, 2 * j + 1]
    return tl, tr, bl, br


DOWNSAMPLES = ("checkerboard", "quad")


def training_pairs(x_std: np.ndarray, downsample: str = "checkerboard"):
    """The four (input, target) pairs of one epoch, in table order.

    checkerboard: the Methods table, up-even -> up-odd, up-odd -> up-even,
    left-even -> left-odd, left-odd -> left-even.
    quad: the paper does not say how its four 2x2-block images are paired.
    Reading: the two diagonals of a block, both ways: TL -> BR, BR -> TL,
    TR -> BL, BL -> TR.  Input and target of a pair then sit at a shared
    block corner, and an epoch still has four steps.
    """
    if downsample == "checkerboard":
        ue, uo = checkerboard_up(x_std)
        le, lo = checkerboard_left(x_std)
        return [(ue, uo), (uo, ue), (le, lo), (lo, le)]
    if downsample == "quad":
        tl, tr, bl, br = quad_downsample(x_std)
        return [(tl, br), (br, tl), (tr, bl), (bl, tr)]
    raise ValueError(f"unknown downsample {downsample!r}")


def exact_pairs(x_std: np.ndarray, s_std: np.ndarray, downsample: str = "checkerboard"):
    """Training pairs of the "Exact" ablation (Methods, Ablation Study;
    Table 1), which needs the clean image.

    The downsampling argument of the Theoretical Background writes a pair's
    target as s_in + n_tgt + (s_tgt - s_in) and drops the last term as small
    (the ODD approximation).  The ablation removes that term from the
    target with the known signal, so the target becomes
    x_tgt - (s_tgt - s_in) = s_in + n_tgt.  Reading: s_std is the clean image
    under the same affine standardisation as the noisy input (the noisy
    image's minimum and maximum), so that the term is in the target's units.
    """
    px = training_pairs(x_std, downsample)
    ps = training_pairs(s_std, downsample)
    return [(xa, xb - (sb - sa)) for (xa, xb), (sa, sb) in zip(px, ps)]


# ---------------------------------------------------------------------------
# Network (Methods, network paragraph)
# ---------------------------------------------------------------------------
def conv3x3(a: np.ndarray, Wt: np.ndarray, b: np.ndarray) -> np.ndarray:
    """'Same' 3x3 cross-correlation with zero padding plus bias.

    out[o, i, j] = b[o] + sum_{c, u, v} W[o, c, u, v] * a[c, i + u - 1, j + v - 1],
    taken tap by tap as a (Cout x Cin) @ (Cin x HW) product.
    """
    Cin, H, W = a.shape
    ap = np.pad(a, ((0, 0), (1, 1), (1, 1)))
    out = np.empty((Wt.shape[0], H * W), dtype=np.float64)
    out[:] = b[:, None]
    for u in range(3):
        for v in range(3):
            out += np.ascontiguousarray(Wt[:, :, u, v]) @ ap[:, u:u + H, v:v + W].reshape(Cin, H * W)
    return out.reshape(Wt.shape[0], H, W)


def conv3x3_backward(a: np.ndarray, Wt: np.ndarray, delta: np.ndarray, need_dx: bool = True):
    """Adjoint of `conv3x3` for an upstream gradient `delta` (Cout, H, W).

    dW[o, c, u, v] = sum_{i, j} delta[o, i, j] * a[c, i + u - 1, j + v - 1]
    db[o]          = sum_{i, j} delta[o, i, j]
    da[c, y, x]    = sum_{o, u, v} W[o, c, u, v] * delta[o, y - u + 1, x - v + 1]
    """
    Cin, H, W = a.shape
    Cout = Wt.shape[0]
    ap = np.pad(a, ((0, 0), (1, 1), (1, 1)))
    d2 = delta.reshape(Cout, H * W)
    dW = np.empty_like(Wt, dtype=np.float64)
    for u in range(3):
        for v in range(3):
            dW[:, :, u, v] = d2 @ ap[:, u:u + H, v:v + W].reshape(Cin, H * W).T
    db = d2.sum(axis=1)
    da = None
    if need_dx:
        dap = np.zeros((Cin, H + 2, W + 2), dtype=np.float64)
        for u in range(3):
            for v in range(3):
                dap[:, u:u + H, v:v + W] += (np.ascontiguousarray(Wt[:, :, u, v]).T @ d2).reshape(Cin, H, W)
        da = dap[:, 1:H + 1, 1:W + 1].copy()
    return dW, db, da


def relu(z: np.ndarray) -> np.ndarray:
    return np.maximum(z, 0.0)


def sigmoid(z: np.ndarray) -> np.ndarray:
    """1 / (1 + exp(-z)), evaluated without overflow for either sign of z."""
    z = np.asarray(z, np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def forward(params: dict, x: np.ndarray, n_layers: int = N_LAYERS):
    """Network output for input x (Cin, H, W).

    Returns (acts, z, y): acts[0] = x, acts[l] = ReLU(conv_l(acts[l-1])) for
    l = 1..n_layers; z = 1x1 head logit (H, W); y = sigmoid(z).
    """
    acts = [np.asarray(x, np.float64)]
    for l in range(1, n_layers + 1):
        acts.append(relu(conv3x3(acts[-1], params[f"W{l}"], params[f"b{l}"])))
    w9 = params[f"W{n_layers + 1}"][0, :, 0, 0]
    b9 = params[f"b{n_layers + 1}"][0]
    z = np.tensordot(w9, acts[-1], axes=(0, 0)) + b9
    return acts, z, sigmoid(z)


def bce_loss(z: np.ndarray, t: np.ndarray) -> float:
    """Mean BCE of sigmoid(z) against target t, in logit form.

    -[t log s + (1 - t) log(1 - s)] with s = sigmoid(z) equals
    softplus(z) - t z; the mean runs over the target's pixels.
    """
    return float(np.mean(np.logaddexp(0.0, z) - t * z))


def bce_grad(z: np.ndarray, t: np.ndarray) -> np.ndarray:
    """d(mean BCE)/dz = (sigmoid(z) - t) / P, P = number of target pixels."""
    return (sigmoid(z) - t) / z.size


def backward(params: dict, acts: list, dz: np.ndarray, n_layers: int = N_LAYERS) -> dict:
    """Gradients of the loss for every parameter, given dL/dz of the head.

    The ReLU derivative is taken as 1 where the activation is positive and 0
    elsewhere (including at 0).
    """
    g = {}
    a_top = acts[n_layers]
    w9 = params[f"W{n_layers + 1}"][0, :, 0, 0]
    g[f"W{n_layers + 1}"] = np.tensordot(a_top, dz, axes=([1, 2], [0, 1])).reshape(1, -1, 1, 1)
    g[f"b{n_layers + 1}"] = np.array([dz.sum()])
    delta = w9[:, None, None] * dz[None] * (a_top > 0)
    for l in range(n_layers, 0, -1):
        dW, db, da = conv3x3_backward(acts[l - 1], params[f"W{l}"], delta, need_dx=(l > 1))
        g[f"W{l}"], g[f"b{l}"] = dW, db
        if l > 1:
            delta = da * (acts[l - 1] > 0)
    return g


# ---------------------------------------------------------------------------
# Adam (Kingma and Ba, Algorithm 1)
# ---------------------------------------------------------------------------
@dataclass
class Hyper:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    patience: int = 100
    max_epochs: int = 2000
    fixed_epochs: int = 0           # > 0: run exactly this many epochs, no early stop
    width: object = WIDTH           # int, or one width per layer (e.g. LITERAL_WIDTHS)
    n_layers: int = N_LAYERS


def adam_step(theta, g, m, v, t, h: Hyper):
    """One Adam update; t is the number of steps taken before this one."""
    t = t + 1
    m = h.beta1 * m + (1.0 - h.beta1) * g
    v = h.beta2 * v + (1.0 - h.beta2) * g * g
    m_hat = m / (1.0 - h.beta1 ** t)
    v_hat = v / (1.0 - h.beta2 ** t)
    theta = theta - h.lr * m_hat / (np.sqrt(v_hat) + h.eps)
    return theta, m, v, t


# ---------------------------------------------------------------------------
# One network's training state and step
# ---------------------------------------------------------------------------
@dataclass
class NetState:
    theta: np.ndarray
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def new_state(theta0: np.ndarray) -> NetState:
    th = np.asarray(theta0, np.float64).copy()
    return NetState(th, np.zeros_like(th), np.zeros_like(th), 0)


def gradients(theta: np.ndarray, C: int, inp: np.ndarray, tgt: np.ndarray, h: Hyper):
    """Loss, flat gradient and output for one (input, target-channel) pair."""
    params = unflatten(theta, C, h.width, h.n_layers)
    acts, z, y = forward(params, inp, h.n_layers)
    loss = bce_loss(z, tgt)
    g = backward(params, acts, bce_grad(z, tgt), h.n_layers)
    return loss, flatten(g, C, h.width, h.n_layers), y


def train_step(st: NetState, C: int, inp: np.ndarray, tgt: np.ndarray, h: Hyper):
    """Forward, BCE, backward and one Adam step (Methods, batch size 1)."""
    loss, g, y = gradients(st.theta, C, inp, tgt, h)
    th, m, v, t = adam_step(st.theta, g, st.m, st.v, st.t, h)
    return NetState(th, m, v, t), g, loss, y


def validate(theta: np.ndarray, C: int, x_std: np.ndarray, k: int, h: Hyper):
    """Full-image output of network k and its MSE against channel k of the
    standardised noisy input, summed in FP64 (Methods, validation)."""
    params = unflatten(theta, C, h.width, h.n_layers)
    _, _, y = forward(params, x_std, h.n_layers)
    return y, float(np.mean((y - x_std[k]) ** 2))


# ---------------------------------------------------------------------------
# Early stopping and output averaging (Methods, validation paragraph)
# ---------------------------------------------------------------------------
@dataclass
class EarlyStop:
    """Running state of the stopping rule.

    After epoch e with score v: a strict improvement (v < best) records the
    epoch and its output and empties the running sum; otherwise the output is
    added to the running sum and counted.  The run ends when `patience`
    epochs in a row did not improve; the result is then the mean of exactly
    those last `patience` outputs.
    """
    patience: int = 100
    best: float = math.inf
    best_epoch: int = 0
    n: int = 0
    S: np.ndarray | None = None
    Y_best: np.ndarray | None = None
    epoch: int = 0
    history: list = field(default_factory=list)

    def update(self, y: np.ndarray, v: float):
        self.epoch += 1
        self.history.append(v)
        if v < self.best:
            self.best, self.best_epoch, self.n = v, self.epoch, 0
            self.Y_best = np.array(y, np.float64, copy=True)
            self.S = np.zeros_like(self.Y_best)
            improved = True
        else:
            self.S = self.S + y
            self.n += 1
            improved = False
        return improved, self.n >= self.patience

    def output(self) -> np.ndarray:
        """Mean of the non-improving outputs since the best epoch, or the best
        output itself when none followed it."""
        if self.n > 0:
            return self.S / self.n
        return self.Y_best


# ---------------------------------------------------------------------------
# Whole loop
# ---------------------------------------------------------------------------
@dataclass
class RunResult:
    y: np.ndarray                      # (C, H, W) output in input units
    y_std: np.ndarray                  # (C, H, W) output in standardised units
    epochs: list                       # per network: epochs run
    best_epoch: list                   # per network
    history: list                      # per network: validation scores
    capped: list                       # per network: stopped by max_epochs
    constant: bool = False


def denoise(x: np.ndarray, theta0: np.ndarray, h: Hyper = Hyper(), pair_order=(0, 1, 2, 3),
            trace=None, downsample: str = "checkerboard", clean=None) -> RunResult:
    """The per-image loop of the paper, one network per output channel.

    x: noisy image (C, H, W); theta0: (C, n_params) initial weights.
    Each epoch feeds the four pairs one at a time (one Adam step each), then
    validates on the full image.  `trace`, if given, is called as
    trace(k, epoch, pair, state, grad, loss) after every step.
    `downsample` picks the pairs (`training_pairs`); a clean image `clean`
    (C, H, W) switches to the targets of the "Exact" ablation
    (`exact_pairs`).  Validation is the same in every variant.
    """
    x = np.asarray(x, np.float64)
    C, H, W = x.shape
    x_std, lo, hi = standardize(x)
    if x_std is None:
        return RunResult(x.copy(), x.copy(), [0] * C, [0] * C, [[] for _ in range(C)], [False] * C, True)
    if clean is None:
        pairs = training_pairs(x_std, downsample)
    else:
        s_std = (np.asarray(clean, np.float64) - lo) / (hi - lo)
        pairs = exact_pairs(x_std, s_std, downsample)
    ys = np.empty((C, H, W))
    epochs, best_e, hist, capped = [], [], [], []
    for k in range(C):
        st = new_state(theta0[k])
        es = EarlyStop(h.patience)
        e = 0
        y_last = None
        while True:
            e += 1
            for p in pair_order:
                inp, tgt = pairs[p]
                st, g, loss, _ = train_step(st, C, inp, tgt[k], h)
                if trace is not None:
                    trace(k, e, p, st, g, loss)
            y_last, v = validate(st.theta, C, x_std, k, h)
            _, done = es.update(y_last, v)
            if h.fixed_epochs > 0:
                if e >= h.fixed_epochs:
                    ys[k] = y_last
                    capped.append(False)
                    break
                continue
            if done:
                ys[k] = es.output()
                capped.append(False)
                break
            if e >= h.max_epochs:
                ys[k] = es.output()
                capped.append(True)
                break
        epochs.append(e)
        best_e.append(es.best_epoch)
        hist.append(list(es.history))
    return RunResult(destandardize(ys, lo, hi), ys, epochs, best_e, hist, capped, False)


# ---------------------------------------------------------------------------
# Volumes (Methods, Fluorescence Microscopy Images: live-cell volumes are
# denoised as individual z-slices and then max projected)
# ---------------------------------------------------------------------------
def max_projection(stack: np.ndarray) -> np.ndarray:
    """Maximum-intensity projection along the first axis (z).

    stack: (Z, ...) with Z >= 1.  A NaN is skipped where another slice holds
    a number (fmax), so only an all-NaN column projects to NaN.
    """
    stack = np.asarray(stack)
    if stack.shape[0] < 1:
        raise ValueError("need at least one slice")
    out = stack[0].copy()
    for z in range(1, stack.shape[0]):
        out = np.fmax(out, stack[z])
    return out


def denoise_volume(stack: np.ndarray, theta0: np.ndarray, h: Hyper = Hyper()):
    """Denoise every z-slice of a (Z, H, W) single-channel stack on its own
    (each with the same initial weights theta0 of shape (1, n_params)), then
    max-project.  Returns (projection, denoised stack)."""
    den = np.stack([denoise(stack[z][None], theta0, h).y[0] for z in range(stack.shape[0])])
    return max_projection(den), den
