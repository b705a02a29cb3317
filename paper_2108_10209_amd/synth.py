"""Seeded synthetic inputs for Noise2Fast workloads.

This module holds no arithmetic of the denoising method itself.  It makes the
inputs that both the GPU library and the CPU reference consume:

* clean test images that stand in for the paper's datasets (the paper uses
  BSD68, Set12, a confocal subset of FMD and its own microscopy, none of which
  are available; see the Results and Methods sections),
* noise models the paper evaluates with (synthetic Gaussian noise, and the
  Gaussian-Poisson noise of fluorescence microscopy, Introduction and Results),
* the random initial network weights, drawn by SplitMix64 (Steele, Lea and
  Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) used
  as a counter-based generator, so that the C++ library can draw the very same
  numbers from the same published definition,
* image-size mixes for the batched and serving workloads, and PSNR.

Every generator takes an explicit seed and uses numpy's PCG64 through a
SeedSequence, so a seed fixes the output on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------------------
# Network shape (the width-64 reading of the Methods section: eight 3x3
# conv+ReLU layers followed by a 1x1 conv and a sigmoid).
# ----------------------------------------------------------------------------
WIDTH = 64
N_LAYERS = 8


LITERAL_WIDTHS = (32, 32, 64, 64, 128, 128, 256, 256)


def param_shapes(C: int, width=WIDTH, n_layers: int = N_LAYERS):
    """Canonical parameter list of one output-channel network.

    Order and shapes of the flat parameter vector exchanged with the library:
    W1 (w1, C, 3, 3), b1 (w1), W2..W8 (w_l, w_{l-1}, 3, 3) with biases, then
    the 1x1 head W9 (1, w8, 1, 1) and b9 (1), with w_l = `width` for every
    layer or `width[l - 1]` when a sequence is given.  Each tensor is
    flattened in C order.  Returns [(name, shape, fan_in)].
    """
    ws = [int(width)] * n_layers if isinstance(width, (int, np.integer)) else [int(v) for v in width]
    assert len(ws) == n_layers
    out = []
    cin = C
    for l in range(1, n_layers + 1):
        wl = ws[l - 1]
        out.append((f"W{l}", (wl, cin, 3, 3), cin * 9))
        out.append((f"b{l}", (wl,), cin * 9))
        cin = wl
    out.append((f"W{n_layers + 1}", (1, cin, 1, 1), cin))
    out.append((f"b{n_layers + 1}", (1,), cin))
    return out


def n_params(C: int, width=WIDTH, n_layers: int = N_LAYERS) -> int:
    return sum(int(np.prod(s)) for _, s, _ in param_shapes(C, width, n_layers))


# ----------------------------------------------------------------------------
# SplitMix64, counter form: output n of stream `seed` is mix(seed + (n+1)*G).
# ----------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 outputs for the given 0-based counters (uint64 array)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix_uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 output."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def init_params(C: int, seed: int, width=WIDTH, n_layers: int = N_LAYERS) -> np.ndarray:
    """Initial weights of the C output-channel networks, shape (C, n_params), FP32.

    Every weight and bias of a layer is drawn from U(-1/sqrt(fan_in),
    +1/sqrt(fan_in)) with fan_in = Cin * kh * kw (the paper leaves the
    initialisation unspecified).  Value of flat index i of network k:
    (2u - 1) * bound in FP64, rounded once to FP32, where u is the SplitMix64
    uniform of counter k * n_params + i.
    """
    npar = n_params(C, width, n_layers)
    out = np.empty((C, npar), dtype=np.float32)
    bounds = np.empty(npar, dtype=np.float64)
    o = 0
    for _, shape, fan_in in param_shapes(C, width, n_layers):
        n = int(np.prod(shape))
        bounds[o:o + n] = 1.0 / math.sqrt(float(fan_in))
        o += n
    for k in range(C):
        cnt = np.arange(npar, dtype=np.uint64) + np.uint64(k * npar)
        u = splitmix_uniform(seed, cnt)
        out[k] = ((2.0 * u - 1.0) * bounds).astype(np.float32)
    return out


# ----------------------------------------------------------------------------
# Clean images
# ----------------------------------------------------------------------------
def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def _minmax01(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    if hi == lo:
        return np.zeros_like(a)
    return (a - lo) / (hi - lo)


def blobs(H: int, W: int, seed: int, C: int = 1) -> np.ndarray:
    """Smooth test scene: 8 Gaussian blobs + 4 hard-edged disks + a gradient.

    Blob centres uniform, widths U(0.04, 0.15) * min(H, W), amplitudes
    U(0.3, 1); disk radii U(0.05, 0.2) * min(H, W), intensities U(0.2, 0.8);
    gradient a*x/W + b*y/H with a, b ~ U(-0.5, 0.5).  Min-max scaled to [0, 1]
    in FP64, returned as FP32 (C, H, W).  For C > 1 the geometry is shared and
    each channel gets amplitude multipliers U(0.5, 1) per component.
    """
    rng = _rng(seed, 101)
    m = float(min(H, W))
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    comps = []
    for _ in range(8):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        sg = rng.uniform(0.04, 0.15) * m
        amp = rng.uniform(0.3, 1.0)
        comps.append(amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sg * sg)))
    for _ in range(4):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        r = rng.uniform(0.05, 0.2) * m
        inten = rng.uniform(0.2, 0.8)
        comps.append(inten * (((yy - cy) ** 2 + (xx - cx) ** 2) <= r * r).astype(np.float64))
    a, b = rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5)
    grad = a * xx / W + b * yy / H
    out = np.empty((C, H, W), dtype=np.float32)
    for c in range(C):
        if c == 0:
            mult = np.ones(len(comps))
        else:
            mult = rng.uniform(0.5, 1.0, size=len(comps))
        img = grad.copy()
        for wgt, comp in zip(mult, comps):
            img += wgt * comp
        out[c] = _minmax01(img).astype(np.float32)
    return out


def microscopy(H: int, W: int, seed: int, n_spots: int = 2000, n_fil: int = 30) -> np.ndarray:
    """Fluorescence-like scene: diffraction-limited spots plus filaments.

    Spots: Gaussian PSF sigma 1.5 px, centres uniform, amplitude U(0.3, 1).
    Filaments: cubic Bezier curves through 4 uniform control points, Gaussian
    cross-section sigma 1 px, intensity U(0.2, 0.6).  Quantised to 16 bits
    (round(65535 * s / max s)) and rescaled by 1/65535.  FP32 (1, H, W).
    """
    rng = _rng(seed, 202)
    img = np.zeros((H, W), dtype=np.float64)
    # spots, each rendered in a local window of +-6 sigma
    sg, r = 1.5, 9
    for _ in range(n_spots):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        amp = rng.uniform(0.3, 1.0)
        y0, y1 = max(0, int(cy) - r), min(H, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(W, int(cx) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        img[y0:y1, x0:x1] += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sg * sg))
    # filaments: the profile at a pixel is the max over curve samples
    fil = np.zeros((H, W), dtype=np.float64)
    sgf, rf = 1.0, 4
    for _ in range(n_fil):
        P = np.stack([rng.uniform(0, H, 4), rng.uniform(0, W, 4)], axis=1)
        inten = rng.uniform(0.2, 0.6)
        length = np.sum(np.hypot(*(np.diff(P, axis=0).T)))
        ts = np.linspace(0.0, 1.0, max(8, int(2 * length)))
        B = ((1 - ts) ** 3)[:, None] * P[0] + (3 * (1 - ts) ** 2 * ts)[:, None] * P[1] \
            + (3 * (1 - ts) * ts ** 2)[:, None] * P[2] + (ts ** 3)[:, None] * P[3]
        dy, dx = np.meshgrid(np.arange(-rf, rf + 1), np.arange(-rf, rf + 1), indexing="ij")
        for cy, cx in B:
            iy, ix = int(round(cy)), int(round(cx))
            ys, xs = iy + dy, ix + dx
            ok = (ys >= 0) & (ys < H) & (xs >= 0) & (xs < W)
            val = inten * np.exp(-((ys - cy) ** 2 + (xs - cx) ** 2) / (2 * sgf * sgf))
            ys, xs, val = ys[ok], xs[ok], val[ok]
            np.maximum.at(fil, (ys, xs), val)
    img += fil
    q = np.round(65535.0 * img / img.max()) / 65535.0
    return q.astype(np.float32)[None]


def _add_patch(vol: np.ndarray, patch: np.ndarray, y0: int, x0: int, zw: np.ndarray) -> None:
    """vol[z, y0:, x0:] += zw[z] * patch for the planes where zw is not tiny."""
    h, w = patch.shape
    for z in np.nonzero(zw > 1e-4)[0]:
        vol[z, y0:y0 + h, x0:x0 + w] += zw[z] * patch


def cell_volume(Z: int, H: int, W: int, seed: int) -> np.ndarray:
    """Two-channel live-cell z-stack, a stand-in for the confocal volumes of
    the paper's time-lapse (1024x1024 slices, 41 planes 0.5 um apart, a
    nuclear and an actin channel).

    round(H*W / 40000) cells (at least 1), centres uniform in x and y and in
    the middle half of z.  Nuclear channel: per cell a Gaussian nucleus
    (sigma_xy U(12, 24) px, sigma_z U(3, 6) planes, amplitude U(0.4, 1)) and
    40 chromatin spots (sigma_xy 2 px, sigma_z 1.5 planes, amplitude
    U(0.2, 0.6)) scattered around its centre with the nucleus' sigmas.  Actin
    channel: per cell 6 cubic Bezier filaments with control points within
    +-3 sigma_xy of the centre, lying in a plane U(-4, 4) planes from it
    (Gaussian z-profile, sigma 1.5 planes), cross-section sigma 1 px,
    intensity U(0.2, 0.6).  Each channel is scaled by its maximum to
    [0, 1].  Returns FP32 (2, Z, H, W).
    """
    rng = _rng(seed, 505)
    vol = np.zeros((2, Z, H, W), dtype=np.float64)
    zz = np.arange(Z, dtype=np.float64)
    n_cells = max(1, int(round(H * W / 40000.0)))

    def gauss_patch(cy, cx, sg):
        r = int(3 * sg) + 1
        y0, y1 = max(0, int(cy) - r), min(H, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(W, int(cx) + r + 1)
        if y0 >= y1 or x0 >= x1:
            return None, 0, 0
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        return np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * sg * sg)), y0, x0

    for _ in range(n_cells):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        cz = rng.uniform(0.25 * (Z - 1), 0.75 * (Z - 1))
        sxy, sz = rng.uniform(12, 24), rng.uniform(3, 6)
        amp = rng.uniform(0.4, 1.0)
        pt, y0, x0 = gauss_patch(cy, cx, sxy)
        if pt is not None:
            _add_patch(vol[0], amp * pt, y0, x0, np.exp(-(zz - cz) ** 2 / (2 * sz * sz)))
        for _ in range(40):
            py, px, pz = rng.normal(cy, sxy), rng.normal(cx, sxy), rng.normal(cz, sz)
            a = rng.uniform(0.2, 0.6)
            pt, y0, x0 = gauss_patch(py, px, 2.0)
            if pt is not None:
                _add_patch(vol[0], a * pt, y0, x0, np.exp(-(zz - pz) ** 2 / (2 * 1.5 * 1.5)))
        for _ in range(6):
            P = np.stack([rng.uniform(cy - 3 * sxy, cy + 3 * sxy, 4), rng.uniform(cx - 3 * sxy, cx + 3 * sxy, 4)],
                         axis=1)
            fz = cz + rng.uniform(-4, 4)
            inten = rng.uniform(0.2, 0.6)
            length = np.sum(np.hypot(*(np.diff(P, axis=0).T)))
            ts = np.linspace(0.0, 1.0, max(8, int(2 * length)))
            B = ((1 - ts) ** 3)[:, None] * P[0] + (3 * (1 - ts) ** 2 * ts)[:, None] * P[1] \
                + (3 * (1 - ts) * ts ** 2)[:, None] * P[2] + (ts ** 3)[:, None] * P[3]
            ylo = max(0, int(np.floor(B[:, 0].min())) - 4)
            yhi = min(H, int(np.ceil(B[:, 0].max())) + 5)
            xlo = max(0, int(np.floor(B[:, 1].min())) - 4)
            xhi = min(W, int(np.ceil(B[:, 1].max())) + 5)
            if ylo >= yhi or xlo >= xhi:
                continue
            patch = np.zeros((yhi - ylo, xhi - xlo))
            d = np.arange(-4, 5)
            dy, dx = np.meshgrid(d, d, indexing="ij")
            ys = np.rint(B[:, 0])[:, None, None].astype(np.int64) + dy[None]
            xs = np.rint(B[:, 1])[:, None, None].astype(np.int64) + dx[None]
            val = inten * np.exp(-((ys - B[:, 0, None, None]) ** 2 + (xs - B[:, 1, None, None]) ** 2) / 2.0)
            ok = (ys >= ylo) & (ys < yhi) & (xs >= xlo) & (xs < xhi)
            np.maximum.at(patch, (ys[ok] - ylo, xs[ok] - xlo), val[ok])
            _add_patch(vol[1], patch, ylo, xlo, np.exp(-(zz - fz) ** 2 / (2 * 1.5 * 1.5)))
    for c in range(2):
        m = vol[c].max()
        if m > 0:
            vol[c] /= m
    return vol.astype(np.float32)


def index_image(C: int, H: int, W: int) -> np.ndarray:
    """Pixel value = its linear CHW index (exact in FP32 below 2**24 pixels)."""
    assert C * H * W < (1 << 24)
    return np.arange(C * H * W, dtype=np.float32).reshape(C, H, W)


# ----------------------------------------------------------------------------
# Noise (never clipped, as the paper states for its own data loading)
# ----------------------------------------------------------------------------
def add_gaussian(clean: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    rng = _rng(seed, 303)
    return (clean.astype(np.float64) + sigma * rng.standard_normal(clean.shape)).astype(np.float32)


def add_poisson_gaussian(clean: np.ndarray, peak: float, sigma: float, seed: int) -> np.ndarray:
    rng = _rng(seed, 404)
    lam = np.maximum(clean.astype(np.float64), 0.0) * peak
    x = rng.poisson(lam).astype(np.float64) / peak + sigma * rng.standard_normal(clean.shape)
    return x.astype(np.float32)


def psnr(y: np.ndarray, clean: np.ndarray) -> float:
    """PSNR with peak 1 (clean images live in [0, 1]); mean over every value."""
    mse = float(np.mean((np.asarray(y, np.float64) - np.asarray(clean, np.float64)) ** 2))
    return 10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf")


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
def single_512(sigma255: float, noise_seed: int, clean_seed: int = 0, size: int = 512):
    """512x512 grayscale blobs scene with Gaussian noise of sigma/255."""
    clean = blobs(size, size, clean_seed)
    return clean, add_gaussian(clean, sigma255 / 255.0, noise_seed)


def small_64(seed: int = 0):
    """64x64 grayscale blobs scene, sigma 25/255."""
    clean = blobs(64, 64, seed)
    return clean, add_gaussian(clean, 25.0 / 255.0, seed + 1)


def batch_sizes(n: int = 64, lo: int = 256, hi: int = 1024, seed: int = 3):
    """Side lengths of a batch of independent images: H, W uniform integers."""
    rng = _rng(seed, 505)
    return [(int(rng.integers(lo, hi + 1)), int(rng.integers(lo, hi + 1))) for _ in range(n)]


def batch_images(n: int = 64, lo: int = 256, hi: int = 1024, seed: int = 3,
                 peak: float = 30.0, sigma: float = 10.0 / 255.0):
    """Independent grayscale images of uneven sizes, Poisson-Gaussian noise."""
    out = []
    for i, (H, W) in enumerate(batch_sizes(n, lo, hi, seed)):
        clean = blobs(H, W, seed * 1000 + i)
        out.append((clean, add_poisson_gaussian(clean, peak, sigma, seed * 1000 + i)))
    return out


@dataclass
class Request:
    rid: int
    arrival: float        # seconds from trace start
    H: int
    W: int
    C: int
    noise: str            # "gauss" or "poisson"
    level: float          # sigma (in [0,1] units) or Poisson peak
    seed: int


def serving_trace(n: int = 2000, rate: float = 1.0, seed: int = 5,
                  lo: int = 128, hi: int = 2048, p_rgb: float = 0.3):
    """Poisson arrivals at `rate` requests/s; sides log-uniform in [lo, hi];
    3 channels with probability p_rgb; noise per request: Gaussian sigma in
    U[10, 50]/255 or Poisson peak U[5, 50], 50/50."""
    rng = _rng(seed, 606)
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        H = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        W = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        C = 3 if rng.uniform() < p_rgb else 1
        if rng.uniform() < 0.5:
            reqs.append(Request(i, t, H, W, C, "gauss", rng.uniform(10, 50) / 255.0, seed * 100000 + i))
        else:
            reqs.append(Request(i, t, H, W, C, "poisson", rng.uniform(5, 50), seed * 100000 + i))
    return reqs


def request_image(req: Request):
    clean = blobs(req.H, req.W, req.seed, C=req.C)
    if req.noise == "gauss":
        noisy = add_gaussian(clean, req.level, req.seed)
    else:
        noisy = add_poisson_gaussian(clean, req.level, 0.0, req.seed)
    return clean, noisy
