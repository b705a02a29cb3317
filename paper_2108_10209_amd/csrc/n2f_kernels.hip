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
// bias and ReLU.  16 threads per pixel, 4 output channels each.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_conv1(const float* __restrict__ in, int C,
                                                  const float* __restrict__ w1, const float* __restrict__ b1,
                                                  void* __restrict__ out, int bf, int h, int w,
                                                  const DevState* st) {
    if (finished(st)) return;
    __shared__ float sw[kTaps * 3 * kWidth + kWidth];
    for (int i = threadIdx.x; i < kTaps * C * kWidth; i += kBlock) sw[i] = w1[i];
    for (int i = threadIdx.x; i < kWidth; i += kBlock) sw[kTaps * 3 * kWidth + i] = b1[i];
    __syncthreads();
    const int q = threadIdx.x & 15;
    const long long npix = (long long)h * w;
    for (int it = 0; it < 4; ++it) {
        const long long p = ((long long)blockIdx.x * 4 + it) * 16 + (threadIdx.x >> 4);
        if (p >= npix) break;
        const int y = (int)(p / w), x = (int)(p - (long long)y * w);
        float a0 = sw[kTaps * 3 * kWidth + 4 * q + 0], a1 = sw[kTaps * 3 * kWidth + 4 * q + 1];
        float a2 = sw[kTaps * 3 * kWidth + 4 * q + 2], a3 = sw[kTaps * 3 * kWidth + 4 * q + 3];
        for (int t = 0; t < kTaps; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
            const float* src = in + ((long long)yy * w + xx) * C;
            for (int c = 0; c < C; ++c) {
                const float v = src[c];
                const float* ww = sw + (t * C + c) * kWidth + 4 * q;
                a0 = fmaf(v, ww[0], a0);
                a1 = fmaf(v, ww[1], a1);
                a2 = fmaf(v, ww[2], a2);
                a3 = fmaf(v, ww[3], a3);
            }
        }
        store4(out, p * kWidth + 4 * q, make_float4(fmaxf(a0, 0.f), fmaxf(a1, 0.f), fmaxf(a2, 0.f), fmaxf(a3, 0.f)),
               bf != 0);
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of the first layer: dW1[t][c][co] = sum_p x[p + off(t)][c]
// * d1[p][co] and db1[co] = sum_p d1[p][co], one partial sum per split of
// 16x16 pixel tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_wgrad1(const float* __restrict__ in, int C,
                                                   const void* __restrict__ dlt, int bf,
                                                   float* __restrict__ part, int h, int w,
                                                   const DevState* st) {
    if (finished(st)) return;
    __shared__ float sx[18 * 18 * 3];
    __shared__ float sd[256 * kWidth];
    const int nW = kTaps * C * kWidth;
    const int n1 = nW + kWidth;
    float acc[7];
#pragma unroll
    for (int r = 0; r < 7; ++r) acc[r] = 0.f;
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
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            const int o = threadIdx.x + r * kBlock;
            if (o < nW) {
                const int t = o / (C * kWidth), c = (o / kWidth) % C, co = o & 63;
                const int dy = t / 3, dx = t % 3;
                float s = 0.f;
                for (int p = 0; p < 256; ++p)
                    s = fmaf(sx[(((p >> 4) + dy) * 18 + (p & 15) + dx) * C + c], sd[p * kWidth + co], s);
                acc[r] += s;
            } else if (o < n1) {
                const int co = o - nW;
                float s = 0.f;
                for (int p = 0; p < 256; ++p) s += sd[p * kWidth + co];
                acc[r] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 7; ++r) {
        const int o = threadIdx.x + r * kBlock;
        if (o < n1) part[(long long)blockIdx.x * n1 + o] = acc[r];
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
            const double zd = (double)z;
            lacc += (zd > 0.0 ? zd : 0.0) + log1p(exp(-fabs(zd))) - (double)t * zd;
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
    }
    if (last_block(&st->cnt_loss)) {
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (unsigned i = 0; i < gridDim.x; ++i) s += lpart[i];
            st->loss = s / (double)npix;
            st->cnt_loss = 0;
        }
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
    if (last_block(&st->cnt_val)) {
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (unsigned i = 0; i < gridDim.x; ++i) s += vpart[i];
            const double v = s / (double)npix;
            DevState S = *st;
            S.epoch += 1;
            S.last_v = v;
            vtrace[S.epoch - 1] = v;
            if (!isfinite(v)) {
                S.nonfinite = 1;
                S.done = 1;
                S.improved = 0;
                S.pending = 0;
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
                S.pending = 1;
                if (S.fixed_epochs > 0) {
                    if (S.epoch >= S.fixed_epochs) S.done = 1;
                } else if (S.n_since >= S.patience) {
                    S.done = 1;
                } else if (S.epoch >= S.max_epochs) {
                    S.done = 1;
                    S.capped = 1;
                }
            }
            S.cnt_val = 0;
            *st = S;
        }
    }
}

// Fold the last validation output into the running sum: a new best empties
// the sum and becomes the best output; otherwise the output is added.
__global__ __launch_bounds__(kBlock) void k_accumulate(const float* __restrict__ y, float* __restrict__ S,
                                                       float* __restrict__ ybest, long long npix, DevState* st) {
    if (!st->pending) return;
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
    if (last_block(&st->cnt_acc)) {
        if (threadIdx.x == 0) {
            st->pending = 0;
            st->cnt_acc = 0;
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
__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ theta, float* __restrict__ m,
                                                 float* __restrict__ v, float* __restrict__ g,
                                                 const float* __restrict__ part, const float* __restrict__ ginj,
                                                 ParamTable pt, float lr, double beta1, double beta2, float eps,
                                                 float* fwd, float* bwd, uint16_t* fwd16, uint16_t* bwd16,
                                                 DevState* st) {
    if (finished(st)) return;
    // 32 parameters per block; 8 lanes per parameter each sum every 8th
    // split, then the 8 lane sums are added in lane order (fixed order,
    // so the result does not depend on scheduling).
    __shared__ float red[8][33];
    const long long t_new = st->t + 1;
    const int p = threadIdx.x & 31, j = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + p;
    if (i < pt.total && !ginj) {
        const int l = layer_of(pt, i);
        const int il = i - pt.off[l];
        const float* pp = part + pt.poff[l] + il;
        float s = 0.f;
        for (int sp = j; sp < pt.split[l]; sp += 8) s += pp[(long long)sp * pt.n[l]];
        red[j][p] = s;
    }
    __syncthreads();
    if (j == 0 && i < pt.total) {
        const int l = layer_of(pt, i);
        const int il = i - pt.off[l];
        float gi;
        if (ginj) {
            gi = ginj[i];
        } else {
            gi = red[0][p];
#pragma unroll
            for (int k = 1; k < 8; ++k) gi += red[k][p];
        }
        g[i] = gi;
        const float b1 = (float)beta1, b2 = (float)beta2;
        const float bc1 = (float)(1.0 - pow(beta1, (double)t_new));
        const float bc2 = (float)(1.0 - pow(beta2, (double)t_new));
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        const float th = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        m[i] = mi;
        v[i] = vi;
        theta[i] = th;
        if (l >= 1 && l < kLayers && il < kConvW) pack_one(l, il, th, fwd, bwd, fwd16, bwd16);
    }
    if (last_block(&st->cnt_adam)) {
        if (threadIdx.x == 0) {
            st->t = t_new;
            st->cnt_adam = 0;
        }
    }
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
    hipLaunchKernelGGL(k_conv1, dim3(nblocks((long long)h * w, 64)), dim3(kBlock), 0, s, in, C, w1, b1, out, bf16,
                       h, w, st);
    return hipGetLastError();
}

hipError_t launch_wgrad1(const float* in, int C, const void* dlt, float* part, int nsplit, int bf16, int h, int w,
                         const DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_wgrad1, dim3(nsplit), dim3(kBlock), 0, s, in, C, dlt, bf16, part, h, w, st);
    return hipGetLastError();
}

int head_splits(long long npix) {
    long long b = (npix + 255) / 256;
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
    return hipGetLastError();
}

hipError_t launch_accumulate(const float* y, float* S, float* ybest, long long npix, DevState* st,
                             hipStream_t s) {
    const unsigned nb = std::min<unsigned>(nblocks(npix, kBlock * 4), 2048u);
    hipLaunchKernelGGL(k_accumulate, dim3(nb), dim3(kBlock), 0, s, y, S, ybest, npix, st);
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
                       float* bwd, uint16_t* fwd16, uint16_t* bwd16, DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(nblocks(pt.total, 32)), dim3(kBlock), 0, s, theta, m, v, g, part, ginj, pt,
                       lr, beta1, beta2, eps, fwd, bwd, fwd16, bwd16, st);
    return hipGetLastError();
}

hipError_t launch_extract(const float* src, int h, int w, int C, float* out_chw, hipStream_t s) {
    const long long npix = (long long)h * w;
    hipLaunchKernelGGL(k_extract, dim3(nblocks(npix * C, kBlock)), dim3(kBlock), 0, s, src, npix, C, out_chw);
    return hipGetLastError();
}

}  // namespace n2f
