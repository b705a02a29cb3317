"""Per-tensor bar for BF16 gradient parity.

The BF16 path rounds the 64->64 weights, the activations and the deltas to
BF16.  Where a gradient tensor is a near-cancelling sum (a bias gradient late
in training, or any tensor summed over a few pixels of pure noise), that
rounding alone moves it by more than the 2e-2 bar, however the sums are
done.  The test-side estimate used here is the change of the exact FP64
gradient when the 64->64 weights and the stored activations a1..a8 are
rounded to BF16 (the deltas are not); the bar of a tensor is the larger of
2e-2 and twice that change.  The rounding lives in the tests, not in the
oracle: it drives the oracle's own layer functions.
"""
import numpy as np

from oracle import n2f_oracle as O

BF16_BAR = 2e-2


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


def bf16_round(a):
    """Nearest BF16 value, ties to even, as FP64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _rounded_gradient(theta, C, inp, tgt):
    """The exact gradient with the weights of layers 2..8 and each stored
    activation rounded to BF16 (every layer reads the rounded one)."""
    L = O.N_LAYERS
    prm = O.unflatten(theta, C)
    for l in range(2, L + 1):
        prm[f"W{l}"] = bf16_round(prm[f"W{l}"])
    acts = [np.asarray(inp, np.float64)]
    for l in range(1, L + 1):
        acts.append(bf16_round(O.relu(O.conv3x3(acts[-1], prm[f"W{l}"], prm[f"b{l}"]))))
    z = np.tensordot(prm[f"W{L + 1}"][0, :, 0, 0], acts[-1], axes=(0, 0)) + prm[f"b{L + 1}"][0]
    return O.flatten(O.backward(prm, acts, O.bce_grad(z, tgt), L), C)


def bf16_sensitivity(theta, C, inp, tgt, h=O.Hyper()):
    """Per-tensor relative change of the exact gradient under that rounding."""
    _, g, _ = O.gradients(theta, C, inp, tgt, h)
    gb = _rounded_gradient(theta, C, inp, tgt)
    return {nm: rel(a, b) for (nm, a), b in zip(split(gb, C).items(), split(g, C).values())}


def bf16_bars(theta, C, inp, tgt, h=O.Hyper()):
    """Per-tensor bars: max(2e-2, 2 x the weight-rounding change)."""
    return {nm: max(BF16_BAR, 2 * v) for nm, v in bf16_sensitivity(theta, C, inp, tgt, h).items()}
