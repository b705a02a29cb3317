"""FP32 comparisons at ReLU ties.

Where a pre-activation lies within FP32 rounding of zero, an FP32 path may
take that ReLU's decision either way.  Both decisions are correct FP32
results, yet the gradients that follow differ in every tensor below the
tied layer: on a 34x30 three-channel image one unit of the seventh layer,
2e-8 of its layer's RMS away from zero, moves the first layer's weight
gradient by 2e-4 (PyTorch's CPU FP32 convolution moves it the same way).

The oracle stays FP64.  These helpers list the tied units of a state and
evaluate the oracle's own layer functions with a chosen set of those
decisions reversed, so that a test accepts the exact result or the result of
the other decision at a tie, and nothing else.
"""
import itertools

import numpy as np

from oracle import n2f_oracle as O

TIE = 1e-6          # |z| below TIE * rms(z over its layer): within FP32 rounding of zero
MAX_TIES = 6        # tied units whose decisions are enumerated (the tightest ones)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def split(vec, C, width):
    out, o = {}, 0
    for name, shape in O.param_spec(C, width):
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n])
        o += n
    return out


def _forward(prm, inp, L, flips=()):
    """Activations and ReLU decisions, with the decisions of the units in
    `flips` ((layer, flat index) pairs) reversed.  A reversed unit's value is
    its pre-activation where it is switched on and 0 where it is switched
    off; either is within the tie band of 0."""
    acts, masks, zs = [np.asarray(inp, np.float64)], [], []
    for l in range(1, L + 1):
        z = O.conv3x3(acts[-1], prm[f"W{l}"], prm[f"b{l}"])
        m = z > 0
        for fl, idx in flips:
            if fl == l:
                m.flat[idx] = not m.flat[idx]
        zs.append(z)
        masks.append(m)
        acts.append(np.where(m, z, 0.0))
    return acts, masks, zs


def tied_units(theta, C, inp, width, tie=TIE):
    """(margin, layer, flat index) of every tied unit, tightest first."""
    prm = O.unflatten(np.asarray(theta, np.float64), C, width)
    _, _, zs = _forward(prm, inp, O.N_LAYERS)
    out = []
    for l, z in enumerate(zs, start=1):
        r = np.abs(z) / max(np.sqrt(np.mean(z * z)), 1e-300)
        for idx in np.flatnonzero(r.ravel() < tie):
            out.append((float(r.flat[idx]), l, int(idx)))
    return sorted(out)


def gradient_with_flips(theta, C, inp, tgt, width, flips):
    """Flat gradient (canonical layout) of the BCE loss with the ReLU
    decisions of `flips` reversed, from the oracle's conv, head and BCE
    functions; with no flips it is the oracle's gradient."""
    L = O.N_LAYERS
    prm = O.unflatten(np.asarray(theta, np.float64), C, width)
    acts, masks, _ = _forward(prm, inp, L, flips)
    w9 = prm[f"W{L + 1}"][0, :, 0, 0]
    z = np.tensordot(w9, acts[L], axes=(0, 0)) + prm[f"b{L + 1}"][0]
    dz = O.bce_grad(z, tgt)
    g = {f"W{L + 1}": np.tensordot(acts[L], dz, axes=([1, 2], [0, 1])).reshape(1, -1, 1, 1),
         f"b{L + 1}": np.array([dz.sum()])}
    delta = w9[:, None, None] * dz[None] * masks[L - 1]
    for l in range(L, 0, -1):
        dW, db, da = O.conv3x3_backward(acts[l - 1], prm[f"W{l}"], delta, need_dx=(l > 1))
        g[f"W{l}"], g[f"b{l}"] = dW, db
        if l > 1:
            delta = da * masks[l - 2]
    return O.flatten(g, C, width)


def alternatives(theta, C, inp, tgt, width, tie=TIE):
    """(flips, gradient) for every non-empty subset of the tightest tied
    units of this state."""
    units = [(l, i) for _, l, i in tied_units(theta, C, inp, width, tie)[:MAX_TIES]]
    for n in range(1, len(units) + 1):
        for sub in itertools.combinations(units, n):
            yield sub, gradient_with_flips(theta, C, inp, tgt, width, sub)


def fp32_check(g, theta, C, inp, tgt, width, bar=1e-5):
    """Per-tensor check of an FP32 gradient g.  Passes when every tensor is
    within `bar` (norm-wise relative) of the oracle's gradient, or of the
    gradient of one set of reversed decisions at ties.  Returns
    (ok, errors vs the accepted gradient, accepted gradient, flips)."""
    _, g_or, _ = O.gradients(np.asarray(theta, np.float64), C, inp, tgt, O.Hyper(width=width))
    gg = split(g, C, width)

    def errs(ref):
        r = split(ref, C, width)
        return {nm: rel(gg[nm], r[nm]) for nm in gg}

    e = errs(g_or)
    if max(e.values()) < bar:
        return True, e, g_or, ()
    for flips, g_alt in alternatives(theta, C, inp, tgt, width):
        ea = errs(g_alt)
        if max(ea.values()) < bar:
            return True, ea, g_alt, flips
    return False, e, g_or, ()


def fixed_run_outputs(x, theta0, k, h, sens=1e-6):
    """Outputs (input units) of channel k after h.fixed_epochs epochs: the
    oracle's own run, then one run per step at which reversing the tied
    decisions moves some gradient tensor by more than `sens` (that step
    takes the reversed gradient, every other step the exact one).  Steps and
    validation follow the oracle's loop: four pairs in table order, one Adam
    step each, validation after each epoch; the output is the last
    validation's."""
    x = np.asarray(x, np.float64)
    C = x.shape[0]
    xs, lo, hi = O.standardize(x)
    pairs = O.training_pairs(xs)
    sched = [p for _ in range(h.fixed_epochs) for p in range(4)]

    def run(branch=None, g_branch=None):
        st = O.new_state(theta0[k])
        for s, p in enumerate(sched):
            inp, tgt = pairs[p]
            if s == branch:
                th, m, v, t = O.adam_step(st.theta, g_branch, st.m, st.v, st.t, h)
                st = O.NetState(th, m, v, t)
            else:
                st = O.train_step(st, C, inp, tgt[k], h)[0]
            yield s, st

    def output(st):
        y, _ = O.validate(st.theta, C, xs, k, h)
        return O.destandardize(y, lo, hi)

    outs, branches = [], []
    st_prev = O.new_state(theta0[k])
    for s, st in run():
        inp, tgt = pairs[sched[s]]
        units = tied_units(st_prev.theta, C, inp, h.width)
        if units:
            flips = [(l, i) for _, l, i in units[:MAX_TIES]]
            _, g_ex, _ = O.gradients(st_prev.theta, C, inp, tgt[k], h)
            g_fl = gradient_with_flips(st_prev.theta, C, inp, tgt[k], h.width, flips)
            ge, gf = split(g_ex, C, h.width), split(g_fl, C, h.width)
            if max(rel(gf[nm], ge[nm]) for nm in ge) > sens:
                branches.append((s, g_fl))
        st_prev = st
    outs.append(("exact", output(st_prev)))
    for b, g_fl in branches:
        st_b = None
        for _, st_b in run(b, g_fl):
            pass
        outs.append((f"reversed ties at step {b}", output(st_b)))
    return outs
