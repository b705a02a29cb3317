// Networks of any per-layer widths (multiples of 16 up to 256), e.g. the
// Methods' own 32, 32, 64, 64, 128, 128, 256, 256: generic 3x3 convolution,
// weight gradient, heads, Adam and weight packing.  The 64-wide network keeps
// its own tuned kernels (n2f_conv.hip, n2f_kernels.hip); these serve every
// other width.
//
// Every contraction runs on the FP32 matrix cores (16x16x4 MFMA, FP32
// accumulate).  A BF16 run stores its activations, deltas and the weights of
// layers 2..8 as BF16 (round to nearest even) and widens them to FP32 at the
// MFMA: the product of two BF16 values is exact in FP32, so this is the same
// arithmetic as a BF16 MFMA with FP32 accumulation, up to summation order.
// The first layer's weights stay FP32, as on the 64-wide path.
//
// Channels-last activations: pixel p of a C-channel image at [p * C, p * C + C).
// Weight layouts (internal, tap-major): W[t][ci][co] then b[co], t = 3 dy + dx.
// Packed forward operand: fwd[t][ci/4][co][ci%4] for ci < CIpad (zeros past
// Cin); packed data-gradient operand: bwd[t][co/4][ci][co%4] = W[8-t][ci][co]
// (flipped taps, transposed), so the data gradient is the forward kernel.
#include "n2f_internal.h"

#include <algorithm>

namespace n2f {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kT = 16;            // tile side (pixels)
constexpr int kH = kT + 2;        // halo side
constexpr int kKC = 16;           // input channels per staged chunk
constexpr int kHS = kKC + 4;      // LDS floats per staged halo pixel (padded against bank conflicts)

__device__ __forceinline__ bool finished(const DevState* st) { return st != nullptr && st->done; }

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const f32x2_t f = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}
// value rounded to the storage type (BF16: nearest even)
__device__ __forceinline__ void put(float* p, float v) { *p = v; }
__device__ __forceinline__ void put(uint16_t* p, float v) { *p = (uint16_t)pack_bf16x2(v, 0.f); }

// Four consecutive values of a channels-last row, widened to FP32.
__device__ __forceinline__ floatx4 load4f(const float* p) { return *reinterpret_cast<const floatx4*>(p); }
__device__ __forceinline__ floatx4 load4f(const uint16_t* p) {
    const uint2 r = *reinterpret_cast<const uint2*>(p);
    return floatx4{__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u), __uint_as_float(r.y << 16),
                   __uint_as_float(r.y & 0xffff0000u)};
}
__device__ __forceinline__ void store4(float* p, floatx4 v) { *reinterpret_cast<floatx4*>(p) = v; }
__device__ __forceinline__ void store4(uint16_t* p, floatx4 v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
}

// ---------------------------------------------------------------------------
// 3x3 convolution.  MODE 0: out = relu(b + conv(in)), MODE 1 (data gradient):
// out = conv(in) * [act > 0].  Block: 256 threads, a 16x16 pixel tile and 64
// output channels (block z); wave q owns tile rows 4q..4q+3.  The input is
// staged 16 channels at a time as an 18x18 halo in LDS; MFMA rows are
// output channels (weights from the packed operand), columns are the 16
// pixels of a tile row; within each 16-channel chunk the K order is
// permuted identically for both operands (lane group g, step s: channel
// 4g + s), so each lane reads four consecutive channels at once.
// ---------------------------------------------------------------------------
template <class TI, class TW, class TO, int MODE>
__global__ __launch_bounds__(256) void k_gconv(const TI* __restrict__ in, int CI, const TW* __restrict__ wp,
                                               int CIpad, const float* __restrict__ bias,
                                               const TO* __restrict__ act, TO* __restrict__ out, int CO, int h,
                                               int w, const DevState* st) {
    if (finished(st)) return;
    __shared__ __attribute__((aligned(16))) float halo[kH * kH * kHS];
    const int tid = threadIdx.x, lane = tid & 63, wq = tid >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT, co0 = blockIdx.z * 64;
    const int nj = min(4, (CO - co0) / 16);   // valid 16-channel groups of this block
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < CIpad; c0 += kKC) {
        __syncthreads();   // the previous chunk is consumed
        for (int idx = tid; idx < kH * kH * (kKC / 4); idx += 256) {
            const int pix = idx / (kKC / 4), q = idx - pix * (kKC / 4);
            const int hy = pix / kH, hx = pix - hy * kH;
            const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gy >= 0 && gy < h && gx >= 0 && gx < w) {
                const long long base = ((long long)gy * w + gx) * CI;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ci = c0 + 4 * q + e;
                    if (ci < CI) v[e] = to_f(in[base + ci]);
                }
            }
            *reinterpret_cast<floatx4*>(halo + pix * kHS + 4 * q) = v;
        }
        __syncthreads();
        for (int t = 0; t < kTaps; ++t) {
            const int dy = t / 3, dx = t - 3 * (t / 3);
            floatx4 a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[j] = floatx4{0.f, 0.f, 0.f, 0.f};
                if (j < nj) a[j] = load4f(wp + (((long long)t * (CIpad / 4) + c0 / 4 + g) * CO + co0 + 16 * j + n) * 4);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                b[i] = *reinterpret_cast<const floatx4*>(halo + ((4 * wq + i + dy) * kH + n + dx) * kHS + 4 * g);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j >= nj) continue;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j][s], b[i][s], acc[i][j], 0, 0, 0);
                }
        }
    }
    // D row = output channel 16 j + 4 g + r, column = pixel n of tile row 4 wq + i
    const int gx = x0 + n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gy = y0 + 4 * wq + i;
        if (gy >= h || gx >= w) continue;
        const long long p = (long long)gy * w + gx;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= nj) continue;
            const int co = co0 + 16 * j + 4 * g;
            floatx4 v = acc[i][j];
            if (MODE == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r] + bias[co + r], 0.f);
            } else {
                const floatx4 m = load4f(act + p * CO + co);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = m[r] > 0.f ? v[r] : 0.f;
            }
            store4(out + p * CO + co, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][ci][co] = sum_p src[p + off(t)][ci] * d[p][co] and
// db[co] = sum_p d[p][co], one partial per split: block (split s, input
// chunk of 16 channels, output block of 64) accumulates tiles s, s + S, ...
// MFMA rows are the chunk's input channels, columns 16 output channels,
// K = 4 pixels per step; wave q owns output channels co0 + 16 q .. + 15 for
// all nine taps.  The bias gradient is summed by the blocks of input chunk 0.
// ---------------------------------------------------------------------------
template <class TS, class TD>
__global__ __launch_bounds__(256) void k_gwgrad(const TS* __restrict__ src, int CI, const TD* __restrict__ dlt,
                                                int CO, float* __restrict__ part, int h, int w,
                                                const DevState* st) {
    if (finished(st)) return;
    __shared__ __attribute__((aligned(16))) float sh[kH * kH * kKC];   // source halo, 16 channels
    __shared__ __attribute__((aligned(16))) float dt[kT * kT * 64];    // delta tile, 64 channels
    __shared__ float dbs[4][64];
    const int tid = threadIdx.x, lane = tid & 63, wq = tid >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int nsplit = gridDim.x, sp = blockIdx.x;
    const int ci0 = blockIdx.y * kKC, co0 = blockIdx.z * 64;
    const int tiles_x = (w + kT - 1) / kT, tiles_y = (h + kT - 1) / kT, ntiles = tiles_x * tiles_y;
    const bool wave_ok = co0 + 16 * wq < CO;   // this wave's 16 output channels exist
    floatx4 acc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;
    for (int tile = sp; tile < ntiles; tile += nsplit) {
        const int x0 = (tile % tiles_x) * kT, y0 = (tile / tiles_x) * kT;
        __syncthreads();
        for (int idx = tid; idx < kH * kH; idx += 256) {
            const int hy = idx / kH, hx = idx - hy * kH;
            const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
            const bool inside = gy >= 0 && gy < h && gx >= 0 && gx < w;
            const long long base = ((long long)gy * w + gx) * CI;
#pragma unroll
            for (int c = 0; c < kKC; ++c) sh[idx * kKC + c] = (inside && ci0 + c < CI) ? to_f(src[base + ci0 + c]) : 0.f;
        }
        for (int idx = tid; idx < kT * kT * 16; idx += 256) {
            const int p = idx >> 4, q = idx & 15;
            const int gy = y0 + (p >> 4), gx = x0 + (p & 15);
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gy < h && gx < w && co0 + 4 * q < CO) v = load4f(dlt + ((long long)gy * w + gx) * CO + co0 + 4 * q);
            *reinterpret_cast<floatx4*>(dt + p * 64 + 4 * q) = v;
        }
        __syncthreads();
        if (blockIdx.y == 0 && tid < 64) {
            float s = 0.f;
            for (int p = 0; p < kT * kT; ++p) s += dt[p * 64 + tid];
            dbacc += s;
        }
        if (wave_ok) {
            for (int kk = 0; kk < kT * kT / 4; ++kk) {
                const int p = 4 * kk + g;              // this lane group's pixel of the step
                const int py = p >> 4, px = p & 15;
                const float b = dt[p * 64 + 16 * wq + n];
#pragma unroll
                for (int t = 0; t < kTaps; ++t) {
                    const int dy = t / 3, dx = t - 3 * (t / 3);
                    const float a = sh[((py + dy) * kH + px + dx) * kKC + n];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    }
    // D row = input channel ci0 + 4 g + r, column = output channel co0 + 16 wq + n
    const long long nW = (long long)kTaps * CI * CO;
    float* pp = part + (long long)sp * (nW + CO);
    if (wave_ok) {
        const int co = co0 + 16 * wq + n;
#pragma unroll
        for (int t = 0; t < kTaps; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = ci0 + 4 * g + r;
                if (ci < CI) pp[((long long)t * CI + ci) * CO + co] = acc[t][r];
            }
    }
    if (blockIdx.y == 0 && tid < 64 && co0 + tid < CO) pp[nW + co0 + tid] = dbacc;
}

// ---------------------------------------------------------------------------
// Heads on a CI-channel last activation.  16 lanes per pixel, each with
// CI / 16 channels; z is the xor-butterfly sum over the pixel's lanes.
// Training: dL/dz = (sigmoid(z) - t) / P; d8 = dL/dz w9 [a8 > 0]; per block
// partial rows of dW9, db9 and the BCE (FP64).  Validation: the output and
// one FP64 partial of the squared error against the standardised image.
// Block b owns a contiguous range of pixels; sums are fixed-order.
// ---------------------------------------------------------------------------
constexpr int kHeadLanes = 16;
constexpr int kHeadSlots = 256 / kHeadLanes;
constexpr int kHeadMaxC = 256 / kHeadLanes;   // channels per lane at width 256

__device__ __forceinline__ float sum16(float v) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
    return v;
}

template <class TA, bool TRAIN>
__global__ __launch_bounds__(256) void k_ghead(const TA* __restrict__ a8, int CI, const float* __restrict__ tgt,
                                               int C, int k, const float* __restrict__ w9, TA* __restrict__ d8,
                                               float* __restrict__ y, float* __restrict__ part,
                                               double* __restrict__ lpart, long long npix, DevState* st) {
    if (finished(st)) return;
    __shared__ float red[kHeadSlots][257];
    __shared__ double lred[kHeadSlots];
    const int tid = threadIdx.x, ln = tid % kHeadLanes, slot = tid / kHeadLanes;
    const int cpl = CI / kHeadLanes;   // channels per lane (CI is a multiple of 16)
    const long long chunk = (npix + gridDim.x - 1) / gridDim.x;
    const long long p0 = (long long)blockIdx.x * chunk, p1 = min(npix, p0 + chunk);
    const float b9 = w9[CI];
    float hg[kHeadMaxC];
#pragma unroll
    for (int e = 0; e < kHeadMaxC; ++e) hg[e] = 0.f;
    float hb = 0.f;
    double hl = 0.0;
    for (long long p = p0 + slot; p < p1; p += kHeadSlots) {
        float av[kHeadMaxC];
        float zp = 0.f;
#pragma unroll
        for (int e = 0; e < kHeadMaxC; ++e) {
            av[e] = 0.f;
            if (e < cpl) {
                const int c = ln * cpl + e;
                av[e] = to_f(a8[p * CI + c]);
                zp = fmaf(av[e], w9[c], zp);
            }
        }
        const float z = sum16(zp) + b9;
        const float yv = 1.0f / (1.0f + expf(-z));
        const float t = tgt[p * C + k];
        if (!TRAIN) {
            if (ln == 0) {
                y[p] = yv;
                const double e = (double)yv - (double)t;
                hl += e * e;
            }
            continue;
        }
        const float d = (yv - t) / (float)npix;
#pragma unroll
        for (int e = 0; e < kHeadMaxC; ++e) {
            if (e < cpl) {
                const int c = ln * cpl + e;
                put(d8 + p * CI + c, av[e] > 0.f ? d * w9[c] : 0.f);
                hg[e] = fmaf(d, av[e], hg[e]);
            }
        }
        if (ln == 0) {
            hb += d;
            hl += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z);
        }
    }
    if (TRAIN) {
#pragma unroll
        for (int e = 0; e < kHeadMaxC; ++e)
            if (e < cpl) red[slot][ln * cpl + e] = hg[e];
        if (ln == 0) red[slot][CI] = hb;
    }
    if (ln == 0) lred[slot] = hl;
    __syncthreads();
    if (TRAIN) {
        for (int c = tid; c <= CI; c += 256) {
            float s = 0.f;
            for (int q = 0; q < kHeadSlots; ++q) s += red[q][c];
            part[(long long)blockIdx.x * (CI + 1) + c] = s;
        }
    }
    if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < kHeadSlots; ++q) s += lred[q];
        lpart[blockIdx.x] = s;
        if (TRAIN && blockIdx.x == 0) st->t += 1;   // counts the Adam step that follows
    }
}

// ---------------------------------------------------------------------------
// Adam over one network's parameters: the gradient of parameter i is the
// fixed-order sum of its layer's split partials; the last block reports the
// step's loss (fixed-order FP64 sum of the head's partials).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gadam(float* __restrict__ theta, float* __restrict__ m,
                                               float* __restrict__ v, float* __restrict__ g,
                                               const float* __restrict__ part, ParamTable pt, float lr,
                                               double beta1, double beta2, float eps,
                                               const double* __restrict__ lpart, int nloss, long long loss_npix,
                                               DevState* st) {
    if (finished(st)) return;
    if ((int)blockIdx.x == (int)gridDim.x - 1) {
        __shared__ double lred[256];
        double l = 0.0;
        for (int b = threadIdx.x; b < nloss; b += 256) l += lpart[b];
        lred[threadIdx.x] = l;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) lred[threadIdx.x] += lred[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) st->loss = lred[0] / (double)loss_npix;
        return;
    }
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= pt.total) return;
    int l = 0;
    while (l < kLayers && i >= pt.off[l + 1]) ++l;
    const int il = i - pt.off[l];
    const float* pp = part + pt.poff[l] + il;
    float gi = 0.f;
    for (int s = 0; s < pt.split[l]; ++s) gi += pp[(long long)s * pt.n[l]];
    const long long t_new = st->t;
    const float b1 = (float)beta1, b2 = (float)beta2;
    const float omb1 = (float)(1.0 - beta1), omb2 = (float)(1.0 - beta2);
    const float bc1 = (float)(1.0 - pow(beta1, (double)t_new)), bc2 = (float)(1.0 - pow(beta2, (double)t_new));
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    g[i] = gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Packed operands of 3x3 layer l from theta: fwd[t][ci/4][co][ci%4] (ci <
// CIpad, zero past cin) and, for l >= 1, bwd[t][co/4][ci][co%4] =
// W[8 - t][ci][co].
template <class TW>
__global__ __launch_bounds__(256) void k_gpack(const float* __restrict__ theta, int off, int cin, int cout,
                                               int CIpad, TW* __restrict__ fwd, TW* __restrict__ bwd,
                                               const DevState* st) {
    if (finished(st)) return;
    const long long nf = (long long)kTaps * CIpad * cout;
    const long long nb = bwd ? (long long)kTaps * cout * cin : 0;
    for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nf + nb; e += (long long)gridDim.x * 256) {
        if (e < nf) {
            const int r = (int)(e & 3);
            long long q = e >> 2;
            const int co = (int)(q % cout);
            q /= cout;
            const int cb = (int)(q % (CIpad / 4)), t = (int)(q / (CIpad / 4));
            const int ci = 4 * cb + r;
            const float val = ci < cin ? theta[off + ((long long)t * cin + ci) * cout + co] : 0.f;
            put(fwd + e, val);
        } else {
            const long long f = e - nf;
            const int r = (int)(f & 3);
            long long q = f >> 2;
            const int ci = (int)(q % cin);   // output channel of the data gradient
            q /= cin;
            const int cb = (int)(q % (cout / 4)), t = (int)(q / (cout / 4));
            const int co = 4 * cb + r;        // input channel of the data gradient
            put(bwd + f, theta[off + ((long long)(kTaps - 1 - t) * cin + ci) * cout + co]);
        }
    }
}

inline unsigned gblocks(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 4096); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.  bf16 selects BF16 storage of activations and deltas; `first`
// marks the first layer (FP32 image input and FP32 weights).
// ---------------------------------------------------------------------------
hipError_t launch_gconv(const void* in, int CI, bool in_fp32, const void* wp, bool w_fp32, int CIpad,
                        const float* bias, const void* act, void* out, int CO, int mode, int bf16, int h, int w,
                        const DevState* st, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;   // no grouped form
    const dim3 grid((w + kT - 1) / kT, (h + kT - 1) / kT, (CO + 63) / 64);
    if (!bf16) {
        if (mode == 0)
            hipLaunchKernelGGL((k_gconv<float, float, float, 0>), grid, dim3(256), 0, s, (const float*)in, CI,
                               (const float*)wp, CIpad, bias, (const float*)nullptr, (float*)out, CO, h, w, st);
        else
            hipLaunchKernelGGL((k_gconv<float, float, float, 1>), grid, dim3(256), 0, s, (const float*)in, CI,
                               (const float*)wp, CIpad, bias, (const float*)act, (float*)out, CO, h, w, st);
    } else if (in_fp32 && w_fp32) {   // first layer: FP32 image and weights, BF16 activations out
        hipLaunchKernelGGL((k_gconv<float, float, uint16_t, 0>), grid, dim3(256), 0, s, (const float*)in, CI,
                           (const float*)wp, CIpad, bias, (const uint16_t*)nullptr, (uint16_t*)out, CO, h, w, st);
    } else if (mode == 0) {
        hipLaunchKernelGGL((k_gconv<uint16_t, uint16_t, uint16_t, 0>), grid, dim3(256), 0, s, (const uint16_t*)in,
                           CI, (const uint16_t*)wp, CIpad, bias, (const uint16_t*)nullptr, (uint16_t*)out, CO, h, w,
                           st);
    } else {
        hipLaunchKernelGGL((k_gconv<uint16_t, uint16_t, uint16_t, 1>), grid, dim3(256), 0, s, (const uint16_t*)in,
                           CI, (const uint16_t*)wp, CIpad, bias, (const uint16_t*)act, (uint16_t*)out, CO, h, w, st);
    }
    return hipGetLastError();
}

hipError_t launch_gwgrad(const void* src, int CI, bool src_fp32, const void* dlt, int CO, float* part, int nsplit,
                         int bf16, int h, int w, const DevState* st, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;
    const dim3 grid(nsplit, (CI + kKC - 1) / kKC, (CO + 63) / 64);
    if (!bf16)
        hipLaunchKernelGGL((k_gwgrad<float, float>), grid, dim3(256), 0, s, (const float*)src, CI, (const float*)dlt,
                           CO, part, h, w, st);
    else if (src_fp32)
        hipLaunchKernelGGL((k_gwgrad<float, uint16_t>), grid, dim3(256), 0, s, (const float*)src, CI,
                           (const uint16_t*)dlt, CO, part, h, w, st);
    else
        hipLaunchKernelGGL((k_gwgrad<uint16_t, uint16_t>), grid, dim3(256), 0, s, (const uint16_t*)src, CI,
                           (const uint16_t*)dlt, CO, part, h, w, st);
    return hipGetLastError();
}

hipError_t launch_ghead(const void* a8, int CI, const float* tgt, int C, int k, const float* w9, void* d8, float* y,
                        float* part, double* lpart, int nblk, int train, int bf16, long long npix, DevState* st,
                        hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;
    if (CI % kHeadLanes || CI > 256) return hipErrorInvalidValue;
    if (bf16) {
        if (train)
            hipLaunchKernelGGL((k_ghead<uint16_t, true>), dim3(nblk), dim3(256), 0, s, (const uint16_t*)a8, CI, tgt, C,
                               k, w9, (uint16_t*)d8, y, part, lpart, npix, st);
        else
            hipLaunchKernelGGL((k_ghead<uint16_t, false>), dim3(nblk), dim3(256), 0, s, (const uint16_t*)a8, CI, tgt,
                               C, k, w9, (uint16_t*)d8, y, part, lpart, npix, st);
    } else {
        if (train)
            hipLaunchKernelGGL((k_ghead<float, true>), dim3(nblk), dim3(256), 0, s, (const float*)a8, CI, tgt, C, k,
                               w9, (float*)d8, y, part, lpart, npix, st);
        else
            hipLaunchKernelGGL((k_ghead<float, false>), dim3(nblk), dim3(256), 0, s, (const float*)a8, CI, tgt, C, k,
                               w9, (float*)d8, y, part, lpart, npix, st);
    }
    return hipGetLastError();
}

hipError_t launch_gadam(float* theta, float* m, float* v, float* g, const float* part, const ParamTable& pt, float lr,
                        double beta1, double beta2, float eps, const double* lpart, int nloss, long long loss_npix,
                        DevState* st, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;
    const int nblk = (pt.total + 255) / 256 + 1;
    hipLaunchKernelGGL(k_gadam, dim3(nblk), dim3(256), 0, s, theta, m, v, g, part, pt, lr, beta1, beta2, eps, lpart,
                       nloss, loss_npix, st);
    return hipGetLastError();
}

hipError_t launch_gpack(const float* theta, int off, int cin, int cout, int CIpad, void* fwd, void* bwd, bool w_fp32,
                        const DevState* st, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;
    const long long n = (long long)kTaps * CIpad * cout + (bwd ? (long long)kTaps * cout * cin : 0);
    if (w_fp32)
        hipLaunchKernelGGL((k_gpack<float>), dim3(gblocks(n)), dim3(256), 0, s, theta, off, cin, cout, CIpad,
                           (float*)fwd, (float*)bwd, st);
    else
        hipLaunchKernelGGL((k_gpack<uint16_t>), dim3(gblocks(n)), dim3(256), 0, s, theta, off, cin, cout, CIpad,
                           (uint16_t*)fwd, (uint16_t*)bwd, st);
    return hipGetLastError();
}

}  // namespace n2f
