"""Pins of the oracle's data preparation: standardisation and checkerboard
downsampling (Theoretical Background; Methods, implementation details and
Compared Methods), checked against hand-worked values and invariants."""
import json
import os

import numpy as np
import pytest

from oracle import n2f_oracle as O
from paper_2108_10209_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(H, W):
    return (10 * np.arange(H)[:, None] + np.arange(W)[None, :]).astype(np.float64)[None]


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "checkerboard_worked.json")))["cases"])
def test_checkerboard_worked_example(case):
    x = _grid(case["H"], case["W"])
    ue, uo = O.checkerboard_up(x)
    le, lo = O.checkerboard_left(x)
    np.testing.assert_array_equal(ue[0], case["up_even"])
    np.testing.assert_array_equal(uo[0], case["up_odd"])
    np.testing.assert_array_equal(le[0], case["left_even"])
    np.testing.assert_array_equal(lo[0], case["left_odd"])


@pytest.mark.parametrize("H,W", [(4, 4), (6, 8), (3, 5), (5, 4), (7, 9), (2, 2), (64, 64), (33, 17)])
def test_checkerboard_partition_and_parity(H, W):
    """Each pair takes every pixel of the even extent exactly once, and the
    'even' image holds exactly the pixels with row+column even."""
    C = 2
    x = synth.index_image(C, H, W).astype(np.float64)
    Hc, Wc = O.even_extent(H, W)
    for fn in (O.checkerboard_up, O.checkerboard_left):
        e, o = fn(x)
        assert e.shape == o.shape and e.size + o.size == C * Hc * Wc
        ids = np.concatenate([e.ravel(), o.ravel()]).astype(np.int64)
        ref = x[:, :Hc, :Wc].ravel().astype(np.int64)
        np.testing.assert_array_equal(np.sort(ids), np.sort(ref))
        # parity class of every source pixel
        ce = e.astype(np.int64) % (H * W)
        rows, cols = ce // W, ce % W
        assert np.all((rows + cols) % 2 == 0)
        co = o.astype(np.int64) % (H * W)
        assert np.all((co // W + co % W) % 2 == 1)
        # channels are never mixed
        for c in range(C):
            assert np.all(e[c].astype(np.int64) // (H * W) == c)


@pytest.mark.parametrize("H,W", [(4, 6), (8, 8), (5, 7), (10, 3)])
def test_checkerboard_reinterleave(H, W):
    """Putting the pixels back in the checkerboard pattern restores x."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, H, W))
    Hc, Wc = O.even_extent(H, W)
    ue, uo = O.checkerboard_up(x)
    r = np.empty((1, Hc, Wc))
    for i in range(Hc):
        r[0, i, (i % 2)::2] = ue[0, i]
        r[0, i, (1 - i % 2)::2] = uo[0, i]
    np.testing.assert_array_equal(r, x[:, :Hc, :Wc])
    le, lo = O.checkerboard_left(x)
    r2 = np.empty((1, Hc, Wc))
    for j in range(Wc):
        r2[0, (j % 2)::2, j] = le[0, :, j]
        r2[0, (1 - j % 2)::2, j] = lo[0, :, j]
    np.testing.assert_array_equal(r2, x[:, :Hc, :Wc])


@pytest.mark.parametrize("H,W", [(4, 6), (6, 6), (8, 10)])
def test_left_is_transposed_up(H, W):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, H, W))
    le, lo = O.checkerboard_left(x)
    ue_t, uo_t = O.checkerboard_up(np.transpose(x, (0, 2, 1)))
    np.testing.assert_array_equal(le, np.transpose(ue_t, (0, 2, 1)))
    np.testing.assert_array_equal(lo, np.transpose(uo_t, (0, 2, 1)))


def test_training_pairs_table_order():
    x = synth.index_image(1, 6, 8).astype(np.float64)
    pairs = O.training_pairs(x)
    ue, uo = O.checkerboard_up(x)
    le, lo = O.checkerboard_left(x)
    exp = [(ue, uo), (uo, ue), (le, lo), (lo, le)]
    for (a, b), (c, d) in zip(pairs, exp):
        np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(b, d)


def test_standardize_range_and_exact_extremes():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal((3, 17, 11)) * 3 + 1).astype(np.float32)
    xs, lo, hi = O.standardize(x)
    assert lo == float(x.min()) and hi == float(x.max())
    assert xs.min() == 0.0 and xs.max() == 1.0
    # no clipping: values keep their order and spacing (affine map)
    i, j = np.unravel_index(np.argmax(x), x.shape), np.unravel_index(np.argmin(x), x.shape)
    assert xs[i] == 1.0 and xs[j] == 0.0


def test_standardize_affine_invariance():
    """Any positive affine change of units leaves the standardised image
    unchanged (up to rounding), so the method does not depend on units."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 9, 13))
    a, _, _ = O.standardize(x)
    b, _, _ = O.standardize(7.5 * x - 3.0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    y = O.destandardize(a, *O.standardize(x)[1:])
    np.testing.assert_allclose(y, x, atol=1e-14)


def test_standardize_constant_image():
    xs, lo, hi = O.standardize(np.full((1, 4, 4), 0.25))
    assert xs is None and lo == hi == 0.25
    r = O.denoise(np.full((1, 4, 4), 0.25), np.zeros((1, 10)), O.Hyper())
    assert r.constant and np.all(r.y == 0.25)


@pytest.mark.parametrize("sigma255,expect", [(15, 24.61), (25, 20.17), (50, 14.15)])
def test_noise_psnr_closed_form(sigma255, expect):
    """Noisy-input PSNR of unclipped Gaussian noise is 10 log10(1 / sigma^2)."""
    clean = synth.blobs(256, 256, 0)
    noisy = synth.add_gaussian(clean, sigma255 / 255.0, 7)
    assert abs(synth.psnr(noisy, clean) - 10 * np.log10(255.0 ** 2 / sigma255 ** 2)) < 0.05
    assert abs(synth.psnr(noisy, clean) - expect) < 0.05


def test_poisson_noise_statistics():
    clean = np.full((1, 256, 256), 0.5, np.float32)
    x = synth.add_poisson_gaussian(clean, 30.0, 0.0, 3).astype(np.float64) * 30.0
    assert abs(x.mean() - 15.0) < 0.1 and abs(x.var() - 15.0) < 0.3


def test_generators_are_seeded_and_in_range():
    a = synth.blobs(40, 30, 5)
    b = synth.blobs(40, 30, 5)
    np.testing.assert_array_equal(a, b)
    assert a.min() == 0.0 and a.max() == 1.0 and a.dtype == np.float32
    m = synth.microscopy(96, 80, 4, n_spots=50, n_fil=3)
    assert m.shape == (1, 96, 80) and m.min() >= 0 and m.max() == 1.0
    q = np.round(m.astype(np.float64) * 65535.0)
    np.testing.assert_allclose(q, m.astype(np.float64) * 65535.0, atol=2e-3)
    v = synth.cell_volume(9, 120, 100, 2)
    assert v.shape == (2, 9, 120, 100) and v.dtype == np.float32
    assert v.min() >= 0.0 and v[0].max() == 1.0 and v[1].max() == 1.0
    np.testing.assert_array_equal(v, synth.cell_volume(9, 120, 100, 2))
    assert not np.array_equal(v, synth.cell_volume(9, 120, 100, 3))


def test_splitmix64_published_values():
    """SplitMix64 of seed 1234567: first outputs of the published generator
    (Vigna's splitmix64.c), independent of this project's code."""
    z = synth.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    exp = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [int(v) for v in z] == exp


def test_init_params_bounds():
    th = synth.init_params(1, 0)
    assert th.shape == (1, synth.n_params(1)) == (1, 259201)
    o = 0
    for name, shape, fan_in in synth.param_shapes(1):
        n = int(np.prod(shape))
        seg = th[0, o:o + n]
        bound = 1 / np.sqrt(fan_in)
        assert np.all(np.abs(seg) <= bound)
        if n >= 64:
            assert np.abs(seg).max() > 0.9 * bound
        o += n
    assert synth.n_params(3) == 260353


# ---------------------------------------------------------------------------
# Ablations (Methods, Ablation Study; Table 1): 2x2-block downsampling and
# the "Exact" targets
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "quad_worked.json")))["cases"])
def test_quad_worked_example(case):
    tl, tr, bl, br = O.quad_downsample(_grid(case["H"], case["W"]))
    np.testing.assert_array_equal(tl[0], case["tl"])
    np.testing.assert_array_equal(tr[0], case["tr"])
    np.testing.assert_array_equal(bl[0], case["bl"])
    np.testing.assert_array_equal(br[0], case["br"])


@pytest.mark.parametrize("H,W", [(4, 4), (6, 8), (3, 5), (5, 4), (7, 9), (2, 2), (64, 64), (33, 17)])
def test_quad_partition_and_neighbours(H, W):
    """The four images take every pixel of the even extent once; on an index
    image the block neighbours differ by fixed offsets; TL and BR hold the
    checkerboard's even class, TR and BL its odd class."""
    C = 2
    x = synth.index_image(C, H, W).astype(np.float64)
    Hc, Wc = O.even_extent(H, W)
    tl, tr, bl, br = O.quad_downsample(x)
    for a in (tl, tr, bl, br):
        assert a.shape == (C, Hc // 2, Wc // 2)
    ids = np.concatenate([a.ravel() for a in (tl, tr, bl, br)]).astype(np.int64)
    np.testing.assert_array_equal(np.sort(ids), np.sort(x[:, :Hc, :Wc].ravel().astype(np.int64)))
    # index = c*H*W + row*W + col: right neighbour +1, lower neighbour +W
    np.testing.assert_array_equal(tr - tl, np.ones_like(tl))
    np.testing.assert_array_equal(bl - tl, np.full_like(tl, W))
    np.testing.assert_array_equal(br - tl, np.full_like(tl, W + 1))
    # block (i, j) starts at pixel (2i, 2j)
    i, j = np.meshgrid(np.arange(Hc // 2), np.arange(Wc // 2), indexing="ij")
    for c in range(C):
        np.testing.assert_array_equal(tl[c], c * H * W + 2 * i * W + 2 * j)
    ue, uo = O.checkerboard_up(x)
    np.testing.assert_array_equal(np.sort(np.concatenate([tl.ravel(), br.ravel()])), np.sort(ue.ravel()))
    np.testing.assert_array_equal(np.sort(np.concatenate([tr.ravel(), bl.ravel()])), np.sort(uo.ravel()))


def test_quad_training_pairs_are_block_diagonals():
    H, W = 6, 8
    x = synth.index_image(1, H, W).astype(np.float64)
    pairs = O.training_pairs(x, "quad")
    # target minus input on an index image: +-(W+1) along the main diagonal,
    # +-(W-1) along the other one
    offs = [W + 1, -(W + 1), W - 1, -(W - 1)]
    for (a, b), d in zip(pairs, offs):
        assert a.shape == b.shape == (1, H // 2, W // 2)
        np.testing.assert_array_equal(b - a, np.full_like(a, d))
    with pytest.raises(ValueError):
        O.training_pairs(x, "hexagonal")


@pytest.mark.parametrize("downsample", O.DOWNSAMPLES)
def test_exact_targets_are_signal_plus_target_noise(downsample):
    """With x = s + n, the Exact target of a pair is s_in + n_tgt (in the
    standardised units), built here from the parts instead of from x."""
    rng = np.random.default_rng(7)
    C, H, W = 2, 10, 12
    s = rng.uniform(0.0, 1.0, (C, H, W))
    n = 0.1 * rng.standard_normal((C, H, W))
    x = s + n
    x_std, lo, hi = O.standardize(x)
    pairs = O.exact_pairs(x_std, (s - lo) / (hi - lo), downsample)
    s_pairs = O.training_pairs(s, downsample)
    n_pairs = O.training_pairs(n, downsample)
    for (inp, tgt), (s_in, _), (_, n_tgt) in zip(pairs, s_pairs, n_pairs):
        np.testing.assert_allclose(tgt, (s_in - lo) / (hi - lo) + n_tgt / (hi - lo), rtol=0, atol=1e-14)
    # inputs are the noisy image's, untouched
    for (inp, _), (xa, _) in zip(pairs, O.training_pairs(x_std, downsample)):
        np.testing.assert_array_equal(inp, xa)


def test_exact_targets_without_noise_equal_inputs():
    """Noise-free image: the signal difference is all there is, so every
    Exact target is its input."""
    x = synth.index_image(1, 8, 6).astype(np.float64)
    x_std, lo, hi = O.standardize(x)
    for downsample in O.DOWNSAMPLES:
        for a, b in O.exact_pairs(x_std, x_std, downsample):
            np.testing.assert_allclose(b, a, rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# Volumes: z-slices denoised one by one, then max projected (Methods,
# Fluorescence Microscopy Images)
# ---------------------------------------------------------------------------
def _nan(a):
    return np.array([[[np.nan if v is None else v for v in row] for row in sl] for sl in a], dtype=np.float64)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "max_projection_worked.json")))["cases"])
def test_max_projection_worked_example(case):
    got = O.max_projection(_nan(case["stack"]))
    np.testing.assert_array_equal(got, _nan([case["projection"]])[0])


@pytest.mark.parametrize("Z,H,W", [(1, 3, 4), (2, 5, 5), (41, 6, 7), (5, 1, 9)])
def test_max_projection_properties(Z, H, W):
    """The projection bounds every slice from above and is attained at
    every pixel; it does not depend on the slice order."""
    rng = np.random.default_rng(Z * 100 + H + W)
    st = rng.standard_normal((Z, H, W))
    p = O.max_projection(st)
    assert p.shape == (H, W)
    assert np.all(p[None] >= st)
    assert np.all(np.any(p[None] == st, axis=0))
    np.testing.assert_array_equal(O.max_projection(st[rng.permutation(Z)]), p)
    if Z == 1:
        np.testing.assert_array_equal(p, st[0])
    with pytest.raises(ValueError):
        O.max_projection(np.empty((0, H, W)))


def test_denoise_volume_is_slice_by_slice():
    """Each slice of the denoised stack is that slice denoised alone."""
    h = O.Hyper(width=4, n_layers=2, fixed_epochs=2)
    rng = np.random.default_rng(3)
    st = rng.uniform(0, 1, (3, 6, 8))
    spec = O.param_spec(1, h.width, h.n_layers)
    th = np.concatenate([rng.uniform(-0.5, 0.5, int(np.prod(s))) for _, s in spec])[None]
    proj, den = O.denoise_volume(st, th, h)
    for z in range(3):
        np.testing.assert_array_equal(den[z], O.denoise(st[z][None], th, h).y[0])
    np.testing.assert_array_equal(proj, np.max(den, axis=0))
