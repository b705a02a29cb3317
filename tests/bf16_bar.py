"""Per-tensor check of a BF16 gradient against the FP64 oracle.

The BF16 path rounds the 64->64 weights, every stored activation a1..a8 and
every delta to BF16 (round to nearest even) and accumulates in FP32.  Where a
gradient tensor is a near-cancelling sum (a bias gradient late in training,
or any tensor summed over a few pixels of pure noise), that rounding alone
moves it by more than the 2e-2 bar, however the sums are ordered.

`bf16_emulated_gradient` is a test-side model of exactly that rounding: it
drives the oracle's own FP64 layer functions and rounds the weights of layers
2..8, each activation after its ReLU and each delta after its ReLU mask to
BF16, where the kernels do.  The oracle itself stays FP64.

`bf16_check` passes a tensor when its error against the exact gradient is
below 2e-2 (the BF16 bar), or, for an ill-conditioned tensor only (the
model's rounding alone moves it by more than 1e-2), when its error against
the rounding model is below 2e-2.  No bar is widened: the fallback compares
against a tighter reference, not with a larger tolerance.
"""
import numpy as np

from oracle import n2f_oracle as O

BF16_BAR = 2e-2
ILL = 1e-2          # rounding sensitivity above which a tensor counts as ill-conditioned


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def split(vec, C, width=O.WIDTH):
    out, o = {}, 0
    for name, shape in O.param_spec(C, width):
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n])
        o += n
    return out


def bf16_round(a):
    """Nearest BF16 value, ties to even, of the FP32 value of a, as FP64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_emulated_gradient(theta, C, inp, tgt, width=O.WIDTH):
    """Flat gradient with the BF16 path's rounding points applied to the
    oracle's FP64 layer functions (first-layer weights, biases, the head and
    all sums stay unrounded)."""
    L = O.N_LAYERS
    prm = O.unflatten(theta, C, width)
    for l in range(2, L + 1):
        prm[f"W{l}"] = bf16_round(prm[f"W{l}"])
    acts = [np.asarray(inp, np.float64)]
    for l in range(1, L + 1):
        acts.append(bf16_round(O.relu(O.conv3x3(acts[-1], prm[f"W{l}"], prm[f"b{l}"]))))
    w9 = prm[f"W{L + 1}"][0, :, 0, 0]
    z = np.tensordot(w9, acts[L], axes=(0, 0)) + prm[f"b{L + 1}"][0]
    dz = O.bce_grad(z, tgt)
    g = {f"W{L + 1}": np.tensordot(acts[L], dz, axes=([1, 2], [0, 1])).reshape(1, -1, 1, 1),
         f"b{L + 1}": np.array([dz.sum()])}
    delta = bf16_round(w9[:, None, None] * dz[None] * (acts[L] > 0))
    for l in range(L, 0, -1):
        dW, db, da = O.conv3x3_backward(acts[l - 1], prm[f"W{l}"], delta, need_dx=(l > 1))
        g[f"W{l}"], g[f"b{l}"] = dW, db
        if l > 1:
            delta = bf16_round(da * (acts[l - 1] > 0))
    return O.flatten(g, C, width)


def bf16_check(g, theta, C, inp, tgt, h=O.Hyper()):
    """Per-tensor verdict on the GPU gradient g (flat, canonical layout) for
    state theta on one pair.  Returns (ok, rows) with rows[name] = (error vs
    exact, rounding sensitivity, error vs the rounding model, criterion)."""
    _, g_or, _ = O.gradients(theta, C, inp, tgt, h)
    g_em = bf16_emulated_gradient(theta, C, inp, tgt, h.width)
    gg, go, ge = split(g, C, h.width), split(g_or, C, h.width), split(g_em, C, h.width)
    rows, ok = {}, True
    for nm in gg:
        e_exact, sens, e_model = rel(gg[nm], go[nm]), rel(ge[nm], go[nm]), rel(gg[nm], ge[nm])
        if e_exact < BF16_BAR:
            crit = "exact"
        elif sens > ILL and e_model < BF16_BAR:
            crit = "model"
        else:
            crit = "FAIL"
            ok = False
        rows[nm] = (e_exact, sens, e_model, crit)
    return ok, rows


def summary(rows):
    """One line: the worst tensor against the exact gradient, and the
    tensors judged against the rounding model."""
    worst = max(rows, key=lambda nm: rows[nm][0])
    e, s, m, c = rows[worst]
    model = [f"{nm} (exact {rows[nm][0]:.3f}, sens {rows[nm][1]:.3f}, model {rows[nm][2]:.2e})"
             for nm in rows if rows[nm][3] == "model"]
    bad = [nm for nm in rows if rows[nm][3] == "FAIL"]
    return (f"worst vs exact {worst} {e:.2e} (sens {s:.2e}, vs model {m:.2e}); "
            f"judged vs model: {', '.join(model) or 'none'}; failed: {bad or 'none'}")
