// Memory-bound kernels of the Noise2Fast loop on gfx950: min/max,
// standardisation with the checkerboard gather, the first convolution
// (C <= 3 input channels), the 1x1 head with the BCE gradient, the
// validation head with its FP64 MSE and the stopping rule, the running
// output sum, the final output, Adam, and weight packing.
//
// Activations are stored channels-last (pixel-major, 64 channels
// contiguous).  Every per-epoch kernel returns at once if its network is
// already finished, so whole epochs can be queued ahead of the host.
#include "n2f_internal.h"

#include <math.h>

#include <algorithm>

namespace n2f {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ bool finished(const DevState* st) { return st != nullptr && st->done; }

// True in exactly one block: the last of the grid to get here.  Every
// thread's global writes before this call are visible to that block.
__device__ __forceinline__ bool last_block(unsigned* counter) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned nb = gridDim.x * gridDim.y * gridDim.z;
        unsigned prev = atomicAdd(counter, 1u);
        s_last = (prev == nb - 1);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) {              // inf or nan
        return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Load 4 consecutive channels of an activation row as FP32.
__device__ __forceinline__ float4 load4(const void* base, long long idx, bool bf) {
    if (!bf) return *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + idx);
    const uint2 r = *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + idx);
    return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                       __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
}

__device__ __forceinline__ void store4(void* base, long long idx, float4 v, bool bf) {
    if (!bf) {
        *reinterpret_cast<float4*>(reinterpret_cast<float*>(base) + idx) = v;
        return;
    }
    uint2 r;
    r.x = (uint32_t)f32_to_bf16_rne(v.x) | ((uint32_t)f32_to_bf16_rne(v.y) << 16);
    r.y = (uint32_t)f32_to_bf16_rne(v.z) | ((uint32_t)f32_to_bf16_rne(v.w) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + idx) = r;
}

// ---------------------------------------------------------------------------
// Exact min and max of the whole image, with a non-finite flag.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_minmax(const float* __restrict__ x, long long n,
                                                   float* __restrict__ part, unsigned* counter,
                                                   float* __restrict__ lohi, int* nonfinite) {
    __shared__ float smn[kBlock], smx[kBlock];
    float mn = INFINITY, mx = -INFINITY;
    int bad = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const float v = x[i];
        if (!isfinite(v)) {
            bad = 1;
        } else {
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
        }
    }
    if (bad) atomicOr(nonfinite, 1);
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smn[threadIdx.x] = fminf(smn[threadIdx.x], smn[threadIdx.x + s]);
            smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = smn[0];
        part[2 * blockIdx.x + 1] = smx[0];
    }
    if (last_block(counter)) {
        if (threadIdx.x == 0) {
            float a = INFINITY, b = -INFINITY;
            for (unsigned i = 0; i < gridDim.x; ++i) {
                a = fminf(a, part[2 * i]);
                b = fmaxf(b, part[2 * i + 1]);
            }
            lohi[0] = a;
            lohi[1] = b;
            *counter = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Standardise (x - lo) / (hi - lo) in FP64, rounded once to FP32, and scatter
// each pixel of the even extent into its two checkerboard downsamples:
// row+column even -> up-even[i][j/2] and left-even[i/2][j]; odd -> the odd
// pair.  Input CHW; outputs channels-last.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prepare(const float* __restrict__ x, int H, int W, int C,
                                                    const float* __restrict__ lohi, float* __restrict__ xs,
                                                    float* __restrict__ ue, float* __restrict__ uo,
                                                    float* __restrict__ le, float* __restrict__ lo) {
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long hw = (long long)H * W;
    if (idx >= hw * C) return;
    const int c = (int)(idx / hw);
    const long long rem = idx - (long long)c * hw;
    const int i = (int)(rem / W), j = (int)(rem - (long long)i * W);
    const double l = lohi[0], hgh = lohi[1];
    const float v = (float)(((double)x[idx] - l) / (hgh - l));
    xs[rem * C + c] = v;
    const int Hc = H & ~1, Wc = W & ~1;
    if (i < Hc && j < Wc) {
        const long long pu = (long long)i * (Wc >> 1) + (j >> 1);
        const long long pl = (long long)(i >> 1) * Wc + j;
        if (((i + j) & 1) == 0) {
            ue[pu * C + c] = v;
            le[pl * C + c] = v;
        } else {
            uo[pu * C + c] = v;
            lo[pl * C + c] = v;
        }
    }
}

__global__ void k_init_state(DevState* st, int patience, int max_epochs, int fixed_epochs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState s = {};
    s.best = INFINITY;
    s.last_v = 0.0;
    s.patience = patience;
    s.max_epochs = max_epochs;
    s.fixed_epochs = fixed_epochs;
    *st = s;
}

// Internal tap-major index (t, ci, co) of a 64->64 layer to its packed slots.
__device__ __forceinline__ void pack_one(int layer, int il, float val, float* fwd, float* bwd,
                                         uint16_t* fwd16, uint16_t* bwd16) {
    const int t = il >> 12, ci = (il >> 6) & 63, co = il & 63;
    const long long base = (long long)(layer - 1) * kPackN;
    if (fwd) {
        fwd[base + ((t * 16 + (ci >> 2)) * 64 + co) * 4 + (ci & 3)] = val;
        bwd[base + (((8 - t) * 16 + (co >> 2)) * 64 + ci) * 4 + (co & 3)] = val;
    }
    if (fwd16) {
        const uint16_t b = f32_to_bf16_rne(val);
        fwd16[base + ((t * 8 + (ci >> 3)) * 64 + co) * 8 + (ci & 7)] = b;
        bwd16[base + (((8 - t) * 8 + (co >> 3)) * 64 + ci) * 8 + (co & 7)] = b;
    }
}

__device__ __forceinline__ int layer_of(const ParamTable& pt, int i) {
    int l = 0;
#pragma unroll
    for (int k = 1; k <= kLayers; ++k) l += (i >= pt.off[k]) ? 1 : 0;
    return l;
}

__global__ __launch_bounds__(kBlock) void k_pack(const float* __restrict__ theta, ParamTable pt,
                                                 float* fwd, float* bwd, uint16_t* fwd16, uint16_t* bwd16) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= pt.total) return;
    const int l = layer_of(pt, i);
    const int il = i - pt.off[l];
    if (l >= 1 && l < kLayers && il < kConvW) pack_one(l, il, theta[i], fwd, bwd, fwd16, bwd16);
}

// ---------------------------------------------------------------------------
// First 3x3 conv (C <= 3 input channels, K = 9C is too short for MFMA) with
// bias and ReLU.  Thread = (pixel, group of 16 output channels): four
// consecutive lanes write one pixel's 64 channels contiguously.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_conv1(const float* __restrict__ in, int C,
                                                  const float* __restrict__ w1, const float* __restrict__ b1,
                                                  void* __restrict__ out, int bf, int h, int w,
                                                  const DevState* st) {
    if (finished(st)) return;
    __shared__ __attribute__((aligned(16))) float sw[kTaps * 3 * kWidth + kWidth];
    for (int i = threadIdx.x; i < kTaps * C * kWidth; i += kBlock) sw[i] = w1[i];
    for (int i = threadIdx.x; i < kWidth; i += kBlock) sw[kTaps * 3 * kWidth + i] = b1[i];
    __syncthreads();
    const long long p = (long long)blockIdx.x * (kBlock / 4) + (threadIdx.x >> 2);
    const int cg = threadIdx.x & 3;
    if (p >= (long long)h * w) return;
    const int y = (int)(p / w), x = (int)(p - (long long)y * w);
    float acc[16];
    const float4* bb = reinterpret_cast<const float4*>(sw + kTaps * 3 * kWidth + 16 * cg);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float4 v = bb[r];
        acc[4 * r] = v.x;
        acc[4 * r + 1] = v.y;
        acc[4 * r + 2] = v.z;
        acc[4 * r + 3] = v.w;
    }
    for (int t = 0; t < kTaps; ++t) {
        const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
        if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
        const float* src = in + ((long long)yy * w + xx) * C;
        for (int c = 0; c < C; ++c) {
            const float v = src[c];
            const float4* ww = reinterpret_cast<const float4*>(sw + (t * C + c) * kWidth + 16 * cg);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float4 wv = ww[r];
                acc[4 * r] = fmaf(v, wv.x, acc[4 * r]);
                acc[4 * r + 1] = fmaf(v, wv.y, acc[4 * r + 1]);
                acc[4 * r + 2] = fmaf(v, wv.z, acc[4 * r + 2]);
                acc[4 * r + 3] = fmaf(v, wv.w, acc[4 * r + 3]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        store4(out, p * kWidth + 16 * cg + 4 * r,
               make_float4(fmaxf(acc[4 * r], 0.f), fmaxf(acc[4 * r + 1], 0.f), fmaxf(acc[4 * r + 2], 0.f),
                           fmaxf(acc[4 * r + 3], 0.f)),
               bf != 0);
}

// ---------------------------------------------------------------------------
// Weight gradient of the first layer: dW1[t][c][co] = sum_p x[p + off(t)][c]
// * d1[p][co] and db1[co] = sum_p d1[p][co], one partial sum per split of
// 16x16 pixel tiles.  Thread = (output channel, quarter of the tile's
// pixels): the delta read is one distinct word per lane, the input reads
// are wave-wide broadcasts; quarters are added in a fixed order.
// ---------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(kBlock) void k_wgrad1(const float* __restrict__ in,
                                                   const void* __restrict__ dlt, int bf,
                                                   float* __restrict__ part, int h, int w,
                                                   const DevState* st) {
    if (finished(st)) return;
    constexpr int nW = kTaps * C * kWidth;
    constexpr int n1 = nW + kWidth;
    constexpr int nacc = kTaps * C + 1;          // weights (t, c) then the bias
    __shared__ float sx[18 * 18 * C];
    __shared__ float sd[256 * kWidth];
    const int co = threadIdx.x & 63, pg = threadIdx.x >> 6;
    float acc[nacc];
#pragma unroll
    for (int r = 0; r < nacc; ++r) acc[r] = 0.f;
    const int tiles_x = (w + 15) >> 4, tiles_y = (h + 15) >> 4;
    const int ntiles = tiles_x * tiles_y;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * 16, y0 = (tile / tiles_x) * 16;
        for (int i = threadIdx.x; i < 18 * 18 * C; i += kBlock) {
            const int pix = i / C, c = i - pix * C;
            const int gy = y0 - 1 + pix / 18, gx = x0 - 1 + pix % 18;
            sx[i] = (gy >= 0 && gy < h && gx >= 0 && gx < w) ? in[((long long)gy * w + gx) * C + c] : 0.f;
        }
        for (int i = threadIdx.x; i < 256 * 16; i += kBlock) {
            const int p = i >> 4, q = i & 15;
            const int gy = y0 + (p >> 4), gx = x0 + (p & 15);
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (gy < h && gx < w) v = load4(dlt, ((long long)gy * w + gx) * kWidth + 4 * q, bf != 0);
            *reinterpret_cast<float4*>(sd + p * kWidth + 4 * q) = v;
        }
        __syncthreads();
        for (int p = pg * 64; p < pg * 64 + 64; ++p) {
            const float d = sd[p * kWidth + co];
            const int py = p >> 4, px = p & 15;
#pragma unroll
            for (int t = 0; t < kTaps; ++t)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    acc[t * C + c] = fmaf(sx[((py + t / 3) * 18 + px + t % 3) * C + c], d, acc[t * C + c]);
            acc[kTaps * C] += d;
        }
        __syncthreads();
    }
    // add the four pixel quarters in order through LDS (reusing sd)
#pragma unroll
    for (int r = 0; r < nacc; ++r) sd[(pg * nacc + r) * kWidth + co] = acc[r];
    __syncthreads();
    for (int o = threadIdx.x; o < n1; o += kBlock) {
        const int r = (o < nW) ? (o >> 6) : kTaps * C;    // (t * C + c), or the bias slot
        const int c2 = o & 63;
        float s = 0.f;
        for (int q = 0; q < 4; ++q) s += sd[(q * nacc + r) * kWidth + c2];
        part[(long long)blockIdx.x * n1 + o] = s;
    }
}

// ---------------------------------------------------------------------------
// Training head: z = w9 . a8 + b9, y = sigmoid(z), dL/dz = (y - t) / P for
// the mean BCE; d8 = dL/dz * w9 * [a8 > 0]; per-split partial sums of dW9 =
// sum dL/dz * a8, db9 = sum dL/dz, and of the BCE (softplus(z) - t z).
// 16 threads per pixel (4 channels each), 16 pixels per pass.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_head_train(const void* __restrict__ a8, const float* __restrict__ tgt,
                                                       int C, int k, const float* __restrict__ w9,
                                                       const float* __restrict__ b9, void* __restrict__ d8,
                                                       float* __restrict__ part, double* __restrict__ lpart,
                                                       int bf, long long npix, DevState* st) {
    if (finished(st)) return;
    __shared__ float sacc[16][kWidth + 1];
    __shared__ double sl[16];
    const int q = threadIdx.x & 15, pg = threadIdx.x >> 4;
    const float4 wv = *reinterpret_cast<const float4*>(w9 + 4 * q);
    const float bb = *b9;
    const long long chunk = (((npix + gridDim.x - 1) / gridDim.x) + 15) & ~15LL;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = min(npix, p0 + chunk);
    const float invP = 1.0f / (float)npix;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, gb = 0.f;
    double lacc = 0.0;
    for (long long p = p0 + pg; p < p1; p += 16) {
        const float4 a = load4(a8, p * kWidth + 4 * q, bf != 0);
        float z = a.x * wv.x + a.y * wv.y + a.z * wv.z + a.w * wv.w;
        z += __shfl_xor(z, 8, 16);
        z += __shfl_xor(z, 4, 16);
        z += __shfl_xor(z, 2, 16);
        z += __shfl_xor(z, 1, 16);
        z += bb;
        const float y = 1.0f / (1.0f + expf(-z));
        const float t = tgt[p * C + k];
        const float d = (y - t) * invP;
        const float4 dv = make_float4(a.x > 0.f ? d * wv.x : 0.f, a.y > 0.f ? d * wv.y : 0.f,
                                      a.z > 0.f ? d * wv.z : 0.f, a.w > 0.f ? d * wv.w : 0.f);
        store4(d8, p * kWidth + 4 * q, dv, bf != 0);
        g0 = fmaf(d, a.x, g0);
        g1 = fmaf(d, a.y, g1);
        g2 = fmaf(d, a.z, g2);
        g3 = fmaf(d, a.w, g3);
        if (q == 0) {
            gb += d;
            lacc += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z);
        }
    }
    sacc[pg][4 * q + 0] = g0;
    sacc[pg][4 * q + 1] = g1;
    sacc[pg][4 * q + 2] = g2;
    sacc[pg][4 * q + 3] = g3;
    if (q == 0) {
        sacc[pg][kWidth] = gb;
        sl[pg] = lacc;
    }
    __syncthreads();
    if (threadIdx.x <= kWidth) {
        float s = 0.f;
        for (int i = 0; i < 16; ++i) s += sacc[i][threadIdx.x];
        part[(long long)blockIdx.x * kHeadN + threadIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += sl[i];
        lpart[blockIdx.x] = s;
        // one Adam step follows this head: count it (no other block reads t)
        if (blockIdx.x == 0) st->t += 1;
    }
}

// ---------------------------------------------------------------------------
// Validation head: y = sigmoid(w9 . a8 + b9) over the full image, FP64
// partial sums of (y - x_k)^2, and in the last block the score and the
// stopping rule (strict improvement; `patience` non-improving epochs end
// the run; or exactly `fixed_epochs` epochs).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_head_val(const void* __restrict__ a8, const float* __restrict__ xs,
                                                     int C, int k, const float* __restrict__ w9,
                                                     const float* __restrict__ b9, float* __restrict__ y,
                                                     double* __restrict__ vpart, int bf, long long npix,
                                                     DevState* st, double* __restrict__ vtrace) {
    if (finished(st)) return;
    __shared__ double sl[16];
    const int q = threadIdx.x & 15, pg = threadIdx.x >> 4;
    const float4 wv = *reinterpret_cast<const float4*>(w9 + 4 * q);
    const float bb = *b9;
    const long long chunk = (((npix + gridDim.x - 1) / gridDim.x) + 15) & ~15LL;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = min(npix, p0 + chunk);
    double acc = 0.0;
    for (long long p = p0 + pg; p < p1; p += 16) {
        const float4 a = load4(a8, p * kWidth + 4 * q, bf != 0);
        float z = a.x * wv.x + a.y * wv.y + a.z * wv.z + a.w * wv.w;
        z += __shfl_xor(z, 8, 16);
        z += __shfl_xor(z, 4, 16);
        z += __shfl_xor(z, 2, 16);
        z += __shfl_xor(z, 1, 16);
        z += bb;
        if (q == 0) {
            const float yv = 1.0f / (1.0f + expf(-z));
            y[p] = yv;
            const double e = (double)yv - (double)xs[p * C + k];
            acc += e * e;
        }
    }
    if (q == 0) sl[pg] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += sl[i];
        vpart[blockIdx.x] = s;
    }
}

// Score of the last validation (fixed-order FP64 sum of the block partials)
// and the stopping rule: a strict improvement records the epoch; `patience`
// epochs in a row without one end the run; fixed-epoch mode ends after
// `fixed_epochs`.  One block.  `acc` tells the next kernel whether there is
// an output to fold in.
__global__ __launch_bounds__(kBlock) void k_decide(const double* __restrict__ vpart, int nblk, long long npix,
                                                   DevState* st, double* __restrict__ vtrace) {
    __shared__ double sv[kBlock];
    if (st->done) {
        if (threadIdx.x == 0) st->acc = 0;
        return;
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kBlock) s += vpart[i];
    sv[threadIdx.x] = s;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sv[threadIdx.x] += sv[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double v = sv[0] / (double)npix;
    DevState S = *st;
    S.epoch += 1;
    S.last_v = v;
    vtrace[S.epoch - 1] = v;
    if (!isfinite(v)) {
        S.nonfinite = 1;
        S.done = 1;
        S.improved = 0;
        S.acc = 0;
    } else {
        if (v < S.best) {
            S.best = v;
            S.best_epoch = S.epoch;
            S.n_since = 0;
            S.improved = 1;
        } else {
            S.n_since += 1;
            S.improved = 0;
        }
        S.acc = 1;
        if (S.fixed_epochs > 0) {
            if (S.epoch >= S.fixed_epochs) S.done = 1;
        } else if (S.n_since >= S.patience) {
            S.done = 1;
        } else if (S.epoch >= S.max_epochs) {
            S.done = 1;
            S.capped = 1;
        }
    }
    *st = S;
}

// Fold the last validation output into the running sum: a new best empties
// the sum and becomes the best output; otherwise the output is added.
__global__ __launch_bounds__(kBlock) void k_accumulate(const float* __restrict__ y, float* __restrict__ S,
                                                       float* __restrict__ ybest, long long npix,
                                                       const DevState* st) {
    if (!st->acc) return;
    const int improved = st->improved;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < npix; i += (long long)gridDim.x * kBlock) {
        const float v = y[i];
        if (improved) {
            S[i] = 0.f;
            ybest[i] = v;
        } else {
            S[i] += v;
        }
    }
}

// Output of one channel in input units: the mean of the outputs since the
// best epoch (the best output if none), or the last output in fixed mode.
__global__ __launch_bounds__(kBlock) void k_finalize(const float* __restrict__ y, const float* __restrict__ S,
                                                     const float* __restrict__ ybest, const float* __restrict__ lohi,
                                                     float* __restrict__ out, long long npix, const DevState* st) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= npix) return;
    double r;
    if (st->fixed_epochs > 0) r = y[i];
    else if (st->n_since > 0) r = (double)S[i] / (double)st->n_since;
    else r = ybest[i];
    const double l = lohi[0], hgh = lohi[1];
    out[i] = (float)(l + (hgh - l) * r);
}

// ---------------------------------------------------------------------------
// Adam (Kingma and Ba, Algorithm 1) over one network's flat parameters.
// The gradient is the fixed-order sum of the per-split partials (or an
// injected gradient); bias corrections use the device step counter; the
// packed convolution operands are rewritten from the new weights.
// ---------------------------------------------------------------------------
// One Adam update of parameter i with gradient gi.
__device__ __forceinline__ void adam_one(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                                         int i, float gi, float lr, float b1, float b2, float omb1, float omb2,
                                         float bc1, float bc2, float eps, int l, int il, float* fwd, float* bwd,
                                         uint16_t* fwd16, uint16_t* bwd16) {
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    const float th = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    m[i] = mi;
    v[i] = vi;
    theta[i] = th;
    if (l >= 1 && l < kLayers && il < kConvW) pack_one(l, il, th, fwd, bwd, fwd16, bwd16);
}

// Blocks [0, 7 * kAdamBPL) each own 256 consecutive values of one 64->64
// layer and sum that layer's split partials with 16-byte loads (4 split
// groups, added in group order); the remaining blocks own 32 values of the
// first layer or the head (8 split groups).  Either way the sum order is
// fixed.
constexpr int kAdamBPL = (kConvN + 255) / 256;     // blocks per 64->64 layer

__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ theta, float* __restrict__ m,
                                                 float* __restrict__ v, float* __restrict__ g,
                                                 const float* __restrict__ part, const float* __restrict__ ginj,
                                                 ParamTable pt, float lr, double beta1, double beta2, float eps,
                                                 float* fwd, float* bwd, uint16_t* fwd16, uint16_t* bwd16,
                                                 const double* __restrict__ lpart, int nloss, long long loss_npix,
                                                 DevState* st) {
    if (finished(st)) return;
    __shared__ float4 red4[4][64];
    __shared__ float red[8][33];
    const long long t_new = st->t;   // this step, already counted by the head kernel (or the bump)
    if (blockIdx.x == 0 && threadIdx.x == 0 && !ginj) {
        double l = 0.0;
        for (int b = 0; b < nloss; ++b) l += lpart[b];
        st->loss = l / (double)loss_npix;
    }
    // decay factors and their complements formed in FP64, each rounded
    // once: 1 - (float)0.999 would be off by 1e-5 relative
    const float b1 = (float)beta1, b2 = (float)beta2;
    const float omb1 = (float)(1.0 - beta1), omb2 = (float)(1.0 - beta2);
    const float bc1 = (float)(1.0 - pow(beta1, (double)t_new));
    const float bc2 = (float)(1.0 - pow(beta2, (double)t_new));
    const int nconv = (kLayers - 1) * kAdamBPL;
    if ((int)blockIdx.x < nconv) {
        const int l = 1 + blockIdx.x / kAdamBPL;
        const int il0 = (blockIdx.x % kAdamBPL) * 256;
        const int q = threadIdx.x & 63, j = threadIdx.x >> 6;
        const int il = il0 + 4 * q;
        const bool valid = il < kConvN;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid && !ginj) {
            const float4* pp = reinterpret_cast<const float4*>(part + pt.poff[l] + il);
            const int row4 = kConvN / 4;
#pragma unroll 8
            for (int sp = j; sp < pt.split[l]; sp += 4) {
                const float4 x = pp[(long long)sp * row4];
                acc.x += x.x;
                acc.y += x.y;
                acc.z += x.z;
                acc.w += x.w;
            }
        }
        red4[j][q] = acc;
        __syncthreads();
        if (j == 0 && valid) {
            const int i0 = pt.off[l] + il;
            float gg[4];
            if (ginj) {
#pragma unroll
                for (int e = 0; e < 4; ++e) gg[e] = ginj[i0 + e];
            } else {
                const float4 s0 = red4[0][q], s1 = red4[1][q], s2 = red4[2][q], s3 = red4[3][q];
                gg[0] = ((s0.x + s1.x) + s2.x) + s3.x;
                gg[1] = ((s0.y + s1.y) + s2.y) + s3.y;
                gg[2] = ((s0.z + s1.z) + s2.z) + s3.z;
                gg[3] = ((s0.w + s1.w) + s2.w) + s3.w;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                g[i0 + e] = gg[e];
                adam_one(theta, m, v, i0 + e, gg[e], lr, b1, b2, omb1, omb2, bc1, bc2, eps, l, il + e, fwd, bwd,
                         fwd16, bwd16);
            }
        }
        return;
    }
    // first layer (block range 0) and head (range 1), 32 values per block
    const int nb0 = (pt.n[0] + 31) / 32;
    const int rb = blockIdx.x - nconv;
    const int l = (rb < nb0) ? 0 : kLayers;
    const int il_base = (rb < nb0 ? rb : rb - nb0) * 32;
    const int p = threadIdx.x & 31, j = threadIdx.x >> 5;
    const int il = il_base + p;
    const bool valid = il < pt.n[l];
    float sum = 0.f;
    if (valid && !ginj) {
        const float* pp = part + pt.poff[l] + il;
        for (int sp = j; sp < pt.split[l]; sp += 8) sum += pp[(long long)sp * pt.n[l]];
    }
    red[j][p] = sum;
    __syncthreads();
    if (j == 0 && valid) {
        const int i = pt.off[l] + il;
        float gi;
        if (ginj) {
            gi = ginj[i];
        } else {
            gi = red[0][p];
#pragma unroll
            for (int k = 1; k < 8; ++k) gi += red[k][p];
        }
        g[i] = gi;
        adam_one(theta, m, v, i, gi, lr, b1, b2, omb1, omb2, bc1, bc2, eps, l, il, fwd, bwd, fwd16, bwd16);
    }
}

// Count one Adam step (for steps whose gradient does not come from the head).
__global__ void k_bump_step(DevState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && !st->done) st->t += 1;
}

// Channels-last image (h*w pixels x C) to planar CHW.
__global__ __launch_bounds__(kBlock) void k_extract(const float* __restrict__ src, long long npix, int C,
                                                    float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= npix * C) return;
    const int c = (int)(i / npix);
    const long long p = i - (long long)c * npix;
    out[i] = src[p * C + c];
}

inline unsigned nblocks(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_minmax(const float* x, long long n, float* part, int nblk, unsigned* counter, float* lohi,
                         int* nonfinite, hipStream_t s) {
    hipLaunchKernelGGL(k_minmax, dim3(nblk), dim3(kBlock), 0, s, x, n, part, counter, lohi, nonfinite);
    return hipGetLastError();
}

hipError_t launch_prepare(const float* x, int H, int W, int C, const float* lohi, float* xs, float* ue,
                          float* uo, float* le, float* lo, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(nblocks((long long)H * W * C, kBlock)), dim3(kBlock), 0, s, x, H, W, C,
                       lohi, xs, ue, uo, le, lo);
    return hipGetLastError();
}

hipError_t launch_init_state(DevState* st, int patience, int max_epochs, int fixed_epochs, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, patience, max_epochs, fixed_epochs);
    return hipGetLastError();
}

hipError_t launch_pack(const float* theta, const ParamTable& pt, float* fwd, float* bwd, uint16_t* fwd16,
                       uint16_t* bwd16, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(nblocks(pt.total, kBlock)), dim3(kBlock), 0, s, theta, pt, fwd, bwd, fwd16,
                       bwd16);
    return hipGetLastError();
}

hipError_t launch_conv1(const float* in, int C, const float* w1, const float* b1, void* out, int bf16, int h,
                        int w, const DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_conv1, dim3(nblocks((long long)h * w, kBlock / 4)), dim3(kBlock), 0, s, in, C, w1, b1, out, bf16,
                       h, w, st);
    return hipGetLastError();
}

hipError_t launch_wgrad1(const float* in, int C, const void* dlt, float* part, int nsplit, int bf16, int h, int w,
                         const DevState* st, hipStream_t s) {
    if (C == 1) hipLaunchKernelGGL(k_wgrad1<1>, dim3(nsplit), dim3(kBlock), 0, s, in, dlt, bf16, part, h, w, st);
    else if (C == 2) hipLaunchKernelGGL(k_wgrad1<2>, dim3(nsplit), dim3(kBlock), 0, s, in, dlt, bf16, part, h, w, st);
    else hipLaunchKernelGGL(k_wgrad1<3>, dim3(nsplit), dim3(kBlock), 0, s, in, dlt, bf16, part, h, w, st);
    return hipGetLastError();
}

int head_splits(long long npix) {
    long long b = (npix + 127) / 128;
    return (int)std::max(1LL, std::min(b, (long long)kMaxHeadSplit));
}

hipError_t launch_head_train(const void* a8, const float* tgt, int C, int k, const float* w9, const float* b9,
                             void* d8, float* part, double* lpart, int nsplit, int bf16, long long npix,
                             DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_head_train, dim3(nsplit), dim3(kBlock), 0, s, a8, tgt, C, k, w9, b9, d8, part, lpart,
                       bf16, npix, st);
    return hipGetLastError();
}

hipError_t launch_head_val(const void* a8, const float* xs, int C, int k, const float* w9, const float* b9,
                           float* y, double* vpart, int nblk, int bf16, long long npix, DevState* st,
                           double* vtrace, hipStream_t s) {
    hipLaunchKernelGGL(k_head_val, dim3(nblk), dim3(kBlock), 0, s, a8, xs, C, k, w9, b9, y, vpart, bf16, npix, st,
                       vtrace);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(kBlock), 0, s, (const double*)vpart, nblk, npix, st, vtrace);
    return hipGetLastError();
}

hipError_t launch_accumulate(const float* y, float* S, float* ybest, long long npix, DevState* st,
                             hipStream_t s) {
    const unsigned nb = std::min<unsigned>(nblocks(npix, kBlock * 4), 2048u);
    hipLaunchKernelGGL(k_accumulate, dim3(nb), dim3(kBlock), 0, s, y, S, ybest, npix, (const DevState*)st);
    return hipGetLastError();
}

hipError_t launch_finalize(const float* y, const float* S, const float* ybest, const float* lohi, float* out,
                           long long npix, const DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(nblocks(npix, kBlock)), dim3(kBlock), 0, s, y, S, ybest, lohi, out, npix,
                       st);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, float* m, float* v, float* g, const float* part, const float* ginj,
                       const ParamTable& pt, float lr, double beta1, double beta2, float eps, float* fwd,
                       float* bwd, uint16_t* fwd16, uint16_t* bwd16, const double* lpart, int nloss,
                       long long loss_npix, DevState* st, hipStream_t s) {
    if (ginj) {
        hipLaunchKernelGGL(k_bump_step, dim3(1), dim3(64), 0, s, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nblk = (kLayers - 1) * kAdamBPL + (pt.n[0] + 31) / 32 + (pt.n[kLayers] + 31) / 32;
    hipLaunchKernelGGL(k_adam, dim3(nblk), dim3(kBlock), 0, s, theta, m, v, g, part, ginj, pt,
                       lr, beta1, beta2, eps, fwd, bwd, fwd16, bwd16, lpart, nloss, loss_npix, st);
    return hipGetLastError();
}

hipError_t launch_extract(const float* src, int h, int w, int C, float* out_chw, hipStream_t s) {
    const long long npix = (long long)h * w;
    hipLaunchKernelGGL(k_extract, dim3(nblocks(npix * C, kBlock)), dim3(kBlock), 0, s, src, npix, C, out_chw);
    return hipGetLastError();
}

}  // namespace n2f
