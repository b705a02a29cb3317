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

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to BF16 (to nearest, ties to even) and packed, the
// first in bits 0-15: one gfx950 conversion instruction.  For every non-NaN
// FP32 input it gives the same bits as the software rounding (add 0x7fff plus
// the kept LSB, then truncate), denormals and ties included; a NaN stays NaN.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    const f32x2_t f = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) { return (uint16_t)pack_bf16x2(f, 0.f); }

// Cross-lane sums on the VALU (no LDS round trip): x plus its partner lane.
// add_xor8: partner l ^ 8 inside each 16-lane row (DPP rotate by 8);
// add_xor16 / add_xor32: partner l ^ 16 / l ^ 32, from the gfx950 lane swaps
// of a value with itself (the two results are each lane's own value and its
// partner's, in some order; the sum is the same either way).
__device__ __forceinline__ float add_xor8(float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
}
__device__ __forceinline__ float add_xor16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float add_xor32(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
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
    r.x = pack_bf16x2(v.x, v.y);
    r.y = pack_bf16x2(v.z, v.w);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + idx) = r;
}

// Eight consecutive channels of an activation row as FP32: one 16-byte load
// (BF16) or two (FP32).
template <bool BF>
__device__ __forceinline__ void load8(const void* base, long long idx, float (&v)[8]) {
    if constexpr (BF) {
        const uint4 r = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(base) + idx);
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[2 * e] = __uint_as_float(u[e] << 16);
            v[2 * e + 1] = __uint_as_float(u[e] & 0xffff0000u);
        }
    } else {
        const float4* q = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + idx);
        const float4 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    }
}

template <bool BF>
__device__ __forceinline__ void store8(void* base, long long idx, const float (&v)[8]) {
    if constexpr (BF) {
        uint4 r;
        r.x = pack_bf16x2(v[0], v[1]);
        r.y = pack_bf16x2(v[2], v[3]);
        r.z = pack_bf16x2(v[4], v[5]);
        r.w = pack_bf16x2(v[6], v[7]);
        *reinterpret_cast<uint4*>(reinterpret_cast<uint16_t*>(base) + idx) = r;
    } else {
        float4* q = reinterpret_cast<float4*>(reinterpret_cast<float*>(base) + idx);
        q[0] = make_float4(v[0], v[1], v[2], v[3]);
        q[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
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
// pair.  With `quad` (2x2-block ablation) the pixel goes to one image
// instead, at [i/2][j/2]: ue <- top-left, uo <- bottom-right, le <- top-right,
// lo <- bottom-left, so that the pairs (0,1) and (2,3) are the two block
// diagonals.  Input CHW; outputs channels-last.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prepare(const float* __restrict__ x, int H, int W, int C,
                                                    const float* __restrict__ lohi, float* __restrict__ xs,
                                                    float* __restrict__ ue, float* __restrict__ uo,
                                                    float* __restrict__ le, float* __restrict__ lo, int quad) {
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
    if (quad) {
        if (i < Hc && j < Wc) {
            const long long pq = (long long)(i >> 1) * (Wc >> 1) + (j >> 1);
            float* d = (i & 1) ? ((j & 1) ? uo : lo) : ((j & 1) ? le : ue);
            d[pq * C + c] = v;
        }
    } else if (i < Hc && j < Wc) {
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

// "Exact" ablation targets.  On entry t0..t3 hold the clean image's four
// downsamples (standardised like the noisy ones, same order); on exit the
// target of pair p = (a -> b), x_b - (s_b - s_a), with pairs 0: 0 -> 1,
// 1: 1 -> 0, 2: 2 -> 3, 3: 3 -> 2.  n = values per image (pixels x C).
__global__ __launch_bounds__(kBlock) void k_exact_targets(const float* __restrict__ x0,
                                                          const float* __restrict__ x1,
                                                          const float* __restrict__ x2,
                                                          const float* __restrict__ x3, float* t0, float* t1,
                                                          float* t2, float* t3, long long n) {
    const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    const float s0 = t0[e], s1 = t1[e], s2 = t2[e], s3 = t3[e];
    t0[e] = x1[e] - (s1 - s0);
    t1[e] = x0[e] - (s0 - s1);
    t2[e] = x3[e] - (s3 - s2);
    t3[e] = x2[e] - (s2 - s3);
}

// Maximum-intensity projection along z: out[p] = fmax over z of
// st[z * npix + p] (a NaN loses to any number).  V = 4: one thread owns four
// consecutive pixels and reads 16 bytes per slice (npix % 4 == 0, 16-byte
// aligned pointers); V = 1: one pixel per thread.  Consecutive threads read
// consecutive addresses of each slice.
template <int V>
__global__ __launch_bounds__(kBlock) void k_max_project(const float* __restrict__ st, int nz, long long npix,
                                                        float* __restrict__ out) {
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (V == 4) {
        const long long n4 = npix >> 2;
        if (q >= n4) return;
        const float4* s4 = reinterpret_cast<const float4*>(st);
        float4 m = s4[q];
#pragma unroll 4
        for (int z = 1; z < nz; ++z) {
            const float4 v = s4[(long long)z * n4 + q];
            m.x = fmaxf(m.x, v.x);
            m.y = fmaxf(m.y, v.y);
            m.z = fmaxf(m.z, v.z);
            m.w = fmaxf(m.w, v.w);
        }
        reinterpret_cast<float4*>(out)[q] = m;
    } else {
        if (q >= npix) return;
        float m = st[q];
#pragma unroll 4
        for (int z = 1; z < nz; ++z) m = fmaxf(m, st[(long long)z * npix + q]);
        out[q] = m;
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
// bias and ReLU.  Thread = (pixel slot, lane c of the pixel's 8): it owns
// channels 16 j + 4 g + r for g = c / 2, j = 2 (c % 2) + {0, 1}, r < 4, so
// the eight lanes of a pixel write its 64 channels (two 4-channel stores
// each) and, for BF16 training runs, lane c writes byte c of the pixel's
// ReLU bit mask (bit 16 g + 4 j + r, the layout of the BF16 3x3 kernels).
// Each thread first issues the input-tap loads of all its U pixels
// (lane-uniform within a pixel, served by the cache), then computes and
// stores them, so one memory latency covers U pixels.
// ---------------------------------------------------------------------------
constexpr int kPxPerBlock = kBlock / 8;

template <int C>
constexpr int conv1_unroll() { return C == 1 ? 4 : (C == 2 ? 2 : 1); }

template <int C, bool BF>
__device__ __forceinline__ void conv1_block(const float* __restrict__ in_, const float* __restrict__ w1_,
                                            const float* __restrict__ b1_, void* __restrict__ out_,
                                            uint8_t* __restrict__ mbits_, int h, int w, const DevState* st,
                                            const int bid) {
    const N2F_GLOBAL float* __restrict__ in = as_global(in_);
    const N2F_GLOBAL float* __restrict__ w1 = as_global(w1_);
    const N2F_GLOBAL float* __restrict__ b1 = as_global(b1_);
    N2F_GLOBAL void* __restrict__ out = as_global(out_);
    N2F_GLOBAL uint8_t* __restrict__ mbits = as_global(mbits_);
    const int stop = st->done;   // tested once the loads are in flight
    constexpr int U = conv1_unroll<C>();
    __shared__ __attribute__((aligned(16))) float sw[kTaps * C * kWidth + kWidth];
    for (int i = threadIdx.x; i < kTaps * C * kWidth; i += kBlock) sw[i] = w1[i];
    for (int i = threadIdx.x; i < kWidth; i += kBlock) sw[kTaps * C * kWidth + i] = b1[i];
    const long long npix = (long long)h * w;
    const int cl = threadIdx.x & 7;
    const int c0 = 32 * (cl & 1) + 4 * (cl >> 1), c1 = c0 + 16;
    const long long pbase = (long long)bid * (kPxPerBlock * U) + (threadIdx.x >> 3);
    float xv[U][kTaps * C];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long p = pbase + kPxPerBlock * u;
        const int y = (int)(p / w), x = (int)(p - (long long)y * w);
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            const bool inside = p < npix && yy >= 0 && yy < h && xx >= 0 && xx < w;
#pragma unroll
            for (int c = 0; c < C; ++c) xv[u][t * C + c] = inside ? in[((long long)yy * w + xx) * C + c] : 0.f;
        }
    }
    asm volatile("" ::: "memory");
    if (stop) return;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const long long p = pbase + kPxPerBlock * u;
        if (p >= npix) break;
        float4 a0 = *reinterpret_cast<const float4*>(sw + kTaps * C * kWidth + c0);
        float4 a1 = *reinterpret_cast<const float4*>(sw + kTaps * C * kWidth + c1);
#pragma unroll
        for (int tc = 0; tc < kTaps * C; ++tc) {
            const float v = xv[u][tc];
            const float4 u0 = *reinterpret_cast<const float4*>(sw + tc * kWidth + c0);
            const float4 u1 = *reinterpret_cast<const float4*>(sw + tc * kWidth + c1);
            a0.x = fmaf(v, u0.x, a0.x);
            a0.y = fmaf(v, u0.y, a0.y);
            a0.z = fmaf(v, u0.z, a0.z);
            a0.w = fmaf(v, u0.w, a0.w);
            a1.x = fmaf(v, u1.x, a1.x);
            a1.y = fmaf(v, u1.y, a1.y);
            a1.z = fmaf(v, u1.z, a1.z);
            a1.w = fmaf(v, u1.w, a1.w);
        }
        a0 = make_float4(fmaxf(a0.x, 0.f), fmaxf(a0.y, 0.f), fmaxf(a0.z, 0.f), fmaxf(a0.w, 0.f));
        a1 = make_float4(fmaxf(a1.x, 0.f), fmaxf(a1.y, 0.f), fmaxf(a1.z, 0.f), fmaxf(a1.w, 0.f));
        if (!BF) {
            store4(out, p * kWidth + c0, a0, false);
            store4(out, p * kWidth + c1, a1, false);
        } else {
            // each value rounded to BF16 once, for the store and the mask
            const uint32_t pk[4] = {pack_bf16x2(a0.x, a0.y), pack_bf16x2(a0.z, a0.w), pack_bf16x2(a1.x, a1.y),
                                    pack_bf16x2(a1.z, a1.w)};
            uint32_t b[8];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                b[2 * e] = pk[e] & 0xffffu;
                b[2 * e + 1] = pk[e] >> 16;
            }
            uint16_t* o = reinterpret_cast<uint16_t*>(out) + p * kWidth;
            *reinterpret_cast<uint2*>(o + c0) = make_uint2(pk[0], pk[1]);
            *reinterpret_cast<uint2*>(o + c1) = make_uint2(pk[2], pk[3]);
            if (mbits) {
                uint32_t byte = 0;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if ((b[e] & 0x8000u) == 0 && (b[e] & 0x7fffu) != 0) byte |= 1u << e;    // stored value > 0
                mbits[p * 8 + cl] = (uint8_t)byte;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of the first layer: dW1[t][c][co] = sum_p x[p + off(t)][c]
// * d1[p][co] (x zero outside the image) and db1[co] = sum_p d1[p][co], one
// partial sum per block over a contiguous range of pixels.  Thread = (pixel
// slot, group of G output channels): the delta row of a pixel is read with
// 16-byte (8-byte for G = 4) loads by 64/G lanes; the input taps are
// lane-uniform per pixel.  The slots of a wave are summed by a fixed xor
// butterfly, the waves in order through LDS.
// ---------------------------------------------------------------------------
constexpr int kWg1Block = 512;

template <int C, bool BF>
__device__ __forceinline__ void wgrad1_block(const float* __restrict__ in_, const void* __restrict__ dlt_,
                                             float* __restrict__ part_, int h, int w, const DevState* st,
                                             const int bid, const int nb) {
    const N2F_GLOBAL float* __restrict__ in = as_global(in_);
    const N2F_GLOBAL void* __restrict__ dlt = as_global(dlt_);
    N2F_GLOBAL float* __restrict__ part = as_global(part_);
    const int stop = st->done;                   // tested after the loads of the pixel loop
    constexpr int G = (C == 1) ? 8 : 4;          // channels per lane
    constexpr int LPP = kWidth / G;              // lanes per pixel
    constexpr int SLOTS = kWg1Block / LPP;
    constexpr int nacc = kTaps * C + 1;          // weights (t, c) then the bias
    constexpr int n1 = nacc * kWidth;
    __shared__ float red[kWg1Block / 64][n1];
    const int cg = threadIdx.x % LPP, slot = threadIdx.x / LPP;
    const long long npix = (long long)h * w;
    const long long chunk = (npix + nb - 1) / nb;
    const long long p0 = (long long)bid * chunk;
    const long long p1 = min(npix, p0 + chunk);
    float acc[nacc][G];
#pragma unroll
    for (int r = 0; r < nacc; ++r)
#pragma unroll
        for (int e = 0; e < G; ++e) acc[r][e] = 0.f;
    constexpr int U = 4;                         // pixels per slot per batch, loaded before use
    for (long long pb = p0 + slot; pb < p1; pb += (long long)SLOTS * U) {
        float d[U][G], xv[U][kTaps * C];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long p = pb + (long long)SLOTS * u;
            const bool live = p < p1;
            if constexpr (G == 8) {
                if (live) {
                    load8<BF>(dlt, p * kWidth + 8 * cg, d[u]);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) d[u][e] = 0.f;
                }
            } else {
                const float4 v = live ? load4(dlt, p * kWidth + 4 * cg, BF) : make_float4(0.f, 0.f, 0.f, 0.f);
                d[u][0] = v.x; d[u][1] = v.y; d[u][2] = v.z; d[u][3] = v.w;
            }
            const int y = (int)(p / w), x = (int)(p - (long long)y * w);
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
                const bool inside = live && yy >= 0 && yy < h && xx >= 0 && xx < w;
#pragma unroll
                for (int c = 0; c < C; ++c) xv[u][t * C + c] = inside ? in[((long long)yy * w + xx) * C + c] : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int tc = 0; tc < kTaps * C; ++tc)
#pragma unroll
                for (int e = 0; e < G; ++e) acc[tc][e] = fmaf(xv[u][tc], d[u][e], acc[tc][e]);
#pragma unroll
            for (int e = 0; e < G; ++e) acc[kTaps * C][e] += d[u][e];
        }
    }
    asm volatile("" ::: "memory");
    if (stop) return;
    // slots of one wave: lanes cg, cg + LPP, ... hold the same channels
    // (LPP is 8 or 16: an xor butterfly over the remaining lane bits)
#pragma unroll
    for (int r = 0; r < nacc; ++r)
#pragma unroll
        for (int e = 0; e < G; ++e) {
            float v = acc[r][e];
            if (LPP == 8) v = add_xor8(v);
            v = add_xor16(v);
            acc[r][e] = add_xor32(v);
        }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) < LPP) {
#pragma unroll
        for (int r = 0; r < nacc; ++r)
#pragma unroll
            for (int e = 0; e < G; ++e) red[wv][r * kWidth + G * cg + e] = acc[r][e];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < n1; o += kWg1Block) {
        float sum = red[0][o];
#pragma unroll
        for (int q = 1; q < kWg1Block / 64; ++q) sum += red[q][o];
        part[(long long)bid * n1 + o] = sum;
    }
}

// ---------------------------------------------------------------------------
// Training head: z = w9 . a8 + b9, y = sigmoid(z), dL/dz = (y - t) / P for
// the mean BCE; d8 = dL/dz * w9 * [a8 > 0]; per-split partial sums of dW9 =
// sum dL/dz * a8, db9 = sum dL/dz, and of the BCE (softplus(z) - t z).
// 8 lanes per pixel (8 channels each, one 16-byte row chunk), 32 pixels per
// pass; z is the xor-butterfly sum over the pixel's lanes.
// ---------------------------------------------------------------------------
template <bool BF>
__global__ __launch_bounds__(kBlock) void k_head_train(const void* __restrict__ a8, const float* __restrict__ tgt,
                                                       int C, int k, const float* __restrict__ w9,
                                                       const float* __restrict__ b9, void* __restrict__ d8,
                                                       float* __restrict__ part, double* __restrict__ lpart,
                                                       long long npix, DevState* st) {
    // the stop flag is tested after the pixel loop, so its load overlaps the
    // loop's; a stopped network's delta writes are never read
    const int stop = st->done;
    __shared__ float sacc[kPxPerBlock][kWidth + 1];
    __shared__ double sl[kPxPerBlock];
    const int q = threadIdx.x & 7, ps = threadIdx.x >> 3;
    float wv[8];
    {
        const float4 u = *reinterpret_cast<const float4*>(w9 + 8 * q);
        const float4 v = *reinterpret_cast<const float4*>(w9 + 8 * q + 4);
        wv[0] = u.x; wv[1] = u.y; wv[2] = u.z; wv[3] = u.w;
        wv[4] = v.x; wv[5] = v.y; wv[6] = v.z; wv[7] = v.w;
    }
    const float bb = *b9;
    const long long chunk = (((npix + gridDim.x - 1) / gridDim.x) + kPxPerBlock - 1) / kPxPerBlock * kPxPerBlock;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = min(npix, p0 + chunk);
    const float invP = 1.0f / (float)npix;
    float g[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) g[e] = 0.f;
    float gb = 0.f;
    double lacc = 0.0;
    constexpr int U = 4;                         // pixels per thread per batch, loaded before use
    for (long long pb = p0 + ps; pb < p1; pb += kPxPerBlock * U) {
        float a[U][8], tv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long p = pb + kPxPerBlock * u;
            if (p < p1) {
                load8<BF>(a8, p * kWidth + 8 * q, a[u]);
                tv[u] = tgt[p * C + k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long p = pb + kPxPerBlock * u;
            if (p >= p1) break;
            float z = a[u][0] * wv[0];
#pragma unroll
            for (int e = 1; e < 8; ++e) z = fmaf(a[u][e], wv[e], z);
            z += __shfl_xor(z, 4, 8);
            z += __shfl_xor(z, 2, 8);
            z += __shfl_xor(z, 1, 8);
            z += bb;
            const float y = 1.0f / (1.0f + expf(-z));
            const float t = tv[u];
            const float d = (y - t) * invP;
            float dv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) dv[e] = a[u][e] > 0.f ? d * wv[e] : 0.f;
            store8<BF>(d8, p * kWidth + 8 * q, dv);
#pragma unroll
            for (int e = 0; e < 8; ++e) g[e] = fmaf(d, a[u][e], g[e]);
            if (q == 0) {
                gb += d;
                lacc += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z);
            }
        }
    }
    asm volatile("" ::: "memory");
    if (stop) return;
#pragma unroll
    for (int e = 0; e < 8; ++e) sacc[ps][8 * q + e] = g[e];
    if (q == 0) {
        sacc[ps][kWidth] = gb;
        sl[ps] = lacc;
    }
    __syncthreads();
    if (threadIdx.x <= kWidth) {
        float sum = 0.f;
        for (int i = 0; i < kPxPerBlock; ++i) sum += sacc[i][threadIdx.x];
        part[(long long)blockIdx.x * kHeadN + threadIdx.x] = sum;
    }
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int i = 0; i < kPxPerBlock; ++i) sum += sl[i];
        lpart[blockIdx.x] = sum;
        // one Adam step follows this head: count it (no other block reads t)
        if (blockIdx.x == 0) st->t += 1;
    }
}

// ---------------------------------------------------------------------------
// Validation head: y = sigmoid(w9 . a8 + b9) over the full image and FP64
// partial sums of (y - x_k)^2 per block.  Same lane layout and z sum as the
// training head.
// ---------------------------------------------------------------------------
template <bool BF>
__global__ __launch_bounds__(kBlock) void k_head_val(const void* __restrict__ a8, const float* __restrict__ xs,
                                                     int C, int k, const float* __restrict__ w9,
                                                     const float* __restrict__ b9, float* __restrict__ y,
                                                     double* __restrict__ vpart, long long npix,
                                                     const DevState* st) {
    if (finished(st)) return;
    __shared__ double sl[kPxPerBlock];
    const int q = threadIdx.x & 7, ps = threadIdx.x >> 3;
    float wv[8];
    {
        const float4 u = *reinterpret_cast<const float4*>(w9 + 8 * q);
        const float4 v = *reinterpret_cast<const float4*>(w9 + 8 * q + 4);
        wv[0] = u.x; wv[1] = u.y; wv[2] = u.z; wv[3] = u.w;
        wv[4] = v.x; wv[5] = v.y; wv[6] = v.z; wv[7] = v.w;
    }
    const float bb = *b9;
    const long long chunk = (((npix + gridDim.x - 1) / gridDim.x) + kPxPerBlock - 1) / kPxPerBlock * kPxPerBlock;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = min(npix, p0 + chunk);
    double acc = 0.0;
    constexpr int U = 4;
    for (long long pb = p0 + ps; pb < p1; pb += kPxPerBlock * U) {
        float a[U][8], xk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long p = pb + kPxPerBlock * u;
            if (p < p1) {
                load8<BF>(a8, p * kWidth + 8 * q, a[u]);
                xk[u] = xs[p * C + k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long p = pb + kPxPerBlock * u;
            if (p >= p1) break;
            float z = a[u][0] * wv[0];
#pragma unroll
            for (int e = 1; e < 8; ++e) z = fmaf(a[u][e], wv[e], z);
            z += __shfl_xor(z, 4, 8);
            z += __shfl_xor(z, 2, 8);
            z += __shfl_xor(z, 1, 8);
            z += bb;
            if (q == 0) {
                const float yv = 1.0f / (1.0f + expf(-z));
                y[p] = yv;
                const double e = (double)yv - (double)xk[u];
                acc += e * e;
            }
        }
    }
    if (q == 0) sl[ps] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int i = 0; i < kPxPerBlock; ++i) sum += sl[i];
        vpart[blockIdx.x] = sum;
    }
}

// Score of the last validation (fixed-order FP64 sum of the block partials)
// and the stopping rule: a strict improvement records the epoch; `patience`
// epochs in a row without one end the run; fixed-epoch mode ends after
// `fixed_epochs`.  One block.  `acc` tells the next kernel whether there is
// an output to fold in.
__device__ __forceinline__ void decide_block(const double* __restrict__ vpart_, int nblk, long long npix, DevState* st,
                                             double* __restrict__ vtrace_) {
    const N2F_GLOBAL double* __restrict__ vpart = as_global(vpart_);
    N2F_GLOBAL double* __restrict__ vtrace = as_global(vtrace_);
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
__device__ __forceinline__ void accumulate_block(const float* __restrict__ y_, float* __restrict__ S_,
                                                 float* __restrict__ ybest_, long long npix, const DevState* st,
                                                 const int bid, const int nb) {
    const N2F_GLOBAL float* __restrict__ y = as_global(y_);
    N2F_GLOBAL float* __restrict__ S = as_global(S_);
    N2F_GLOBAL float* __restrict__ ybest = as_global(ybest_);
    if (!st->acc) return;
    const int improved = st->improved;
    for (long long i = (long long)bid * kBlock + threadIdx.x; i < npix; i += (long long)nb * kBlock) {
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

// Blocks [0, 7 * kAdamWPL) each own 256 consecutive values of one 64->64
// layer.  Wave k of such a block sums a lane's 4 values over the k-th
// quarter of the layer's split partials, in split order, with 16-byte loads
// (16 in flight); the four quarter sums are then added in quarter order and
// wave 0 applies Adam.  Four waves per chunk keep enough loads in flight to
// cover the memory latency of the partial reads.
// The blocks after those own a few values of the first layer (4 values x 64
// split groups) or of the head (1 value x 256 split groups), whose partials
// are many short rows: a thread sums every G-th row (a few loads, all in
// flight), and the group sums meet in a fixed-order tree.  The last block
// sums the loss partials.  Every sum order is fixed.
constexpr int kAdamWPL = (kConvN + 255) / 256;           // 256-value chunks per 64->64 layer
constexpr int kAdamConvBlocks = (kLayers - 1) * kAdamWPL;
constexpr int kAdamV0 = 4;                               // first layer: values per block
constexpr int kAdamVH = 1;                               // head: values per block

__device__ __forceinline__ void adam_block(float* __restrict__ theta_, float* __restrict__ m_, float* __restrict__ v_,
                                           float* __restrict__ g_, const float* __restrict__ part_,
                                           const float* __restrict__ ginj_, const ParamTable& pt, float lr,
                                           double beta1, double beta2, float eps, float* fwd_, float* bwd_,
                                           uint16_t* fwd16_, uint16_t* bwd16_, const double* __restrict__ lpart_,
                                           int nloss, long long loss_npix, DevState* st, const int bid,
                                           const int nb) {
    N2F_GLOBAL float* __restrict__ theta = as_global(theta_);
    N2F_GLOBAL float* __restrict__ m = as_global(m_);
    N2F_GLOBAL float* __restrict__ v = as_global(v_);
    N2F_GLOBAL float* __restrict__ g = as_global(g_);
    const N2F_GLOBAL float* __restrict__ part = as_global(part_);
    const N2F_GLOBAL float* __restrict__ ginj = as_global(ginj_);
    N2F_GLOBAL float* fwd = as_global(fwd_);
    N2F_GLOBAL float* bwd = as_global(bwd_);
    N2F_GLOBAL uint16_t* fwd16 = as_global(fwd16_);
    N2F_GLOBAL uint16_t* bwd16 = as_global(bwd16_);
    const N2F_GLOBAL double* __restrict__ lpart = as_global(lpart_);
    if (finished(st)) return;
    __shared__ float red[kBlock];
    __shared__ double lred[kBlock];
    const long long t_new = st->t;   // this step, already counted by the head kernel (or the bump)
    if (bid == nb - 1) {
        // the last block only reports the step's loss: fixed-order sum of
        // the head's FP64 partials (strided per thread, then a tree)
        if (ginj) return;
        double l = 0.0;
        for (int b = threadIdx.x; b < nloss; b += kBlock) l += lpart[b];
        lred[threadIdx.x] = l;
        __syncthreads();
        for (int k = kBlock / 2; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) lred[threadIdx.x] += lred[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) st->loss = lred[0] / (double)loss_npix;
        return;
    }
    // decay factors and their complements formed in FP64, each rounded
    // once: 1 - (float)0.999 would be off by 1e-5 relative
    const float b1 = (float)beta1, b2 = (float)beta2;
    const float omb1 = (float)(1.0 - beta1), omb2 = (float)(1.0 - beta2);
    const float bc1 = (float)(1.0 - pow(beta1, (double)t_new));
    const float bc2 = (float)(1.0 - pow(beta2, (double)t_new));
    if (bid < kAdamConvBlocks) {
        const int l = 1 + bid / kAdamWPL;
        const int il = (bid % kAdamWPL) * 256 + 4 * (threadIdx.x & 63);
        const int wq = threadIdx.x >> 6;
        const bool valid = il < kConvN;   // the layer's last chunk is partly empty
        const int i0 = pt.off[l] + il;
        float gg[4] = {0.f, 0.f, 0.f, 0.f};
        if (ginj) {
            if (wq != 0 || !valid) return;
#pragma unroll
            for (int e = 0; e < 4; ++e) gg[e] = ginj[i0 + e];
        } else {
            __shared__ float4 qsum[4][64];
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            if (valid) {
                const float4* pp = reinterpret_cast<const float4*>(part + pt.poff[l] + il);
                const int row4 = kConvN / 4;
                const int S = pt.split[l];
                const int lo = (wq * S) / 4, hi = ((wq + 1) * S) / 4;
#pragma unroll 16
                for (int sp = lo; sp < hi; ++sp) {
                    const float4 x = pp[(long long)sp * row4];
                    acc.x += x.x;
                    acc.y += x.y;
                    acc.z += x.z;
                    acc.w += x.w;
                }
            }
            qsum[wq][threadIdx.x & 63] = acc;
            __syncthreads();
            if (wq != 0 || !valid) return;
            const int ln = threadIdx.x & 63;
            const float4 a = qsum[0][ln], b = qsum[1][ln], c = qsum[2][ln], d = qsum[3][ln];
            gg[0] = ((a.x + b.x) + c.x) + d.x;
            gg[1] = ((a.y + b.y) + c.y) + d.y;
            gg[2] = ((a.z + b.z) + c.z) + d.z;
            gg[3] = ((a.w + b.w) + c.w) + d.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            g[i0 + e] = gg[e];
            adam_one(theta, m, v, i0 + e, gg[e], lr, b1, b2, omb1, omb2, bc1, bc2, eps, l, il + e, fwd, bwd, fwd16,
                     bwd16);
        }
        return;
    }
    // first layer, then the head
    const int nb0 = (pt.n[0] + kAdamV0 - 1) / kAdamV0;
    const int rb = bid - kAdamConvBlocks;
    const bool first = rb < nb0;
    const int l = first ? 0 : kLayers;
    const int V = first ? kAdamV0 : kAdamVH;
    const int G = kBlock / V;
    const int il = (first ? rb : rb - nb0) * V + (int)threadIdx.x % V;
    const int j = (int)threadIdx.x / V;
    const bool valid = il < pt.n[l];
    float sum = 0.f;
    if (valid && !ginj) {
        const float* pp = part + pt.poff[l] + il;
#pragma unroll 4
        for (int sp = j; sp < pt.split[l]; sp += G) sum += pp[(long long)sp * pt.n[l]];
    }
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int half = G / 2; half > 0; half >>= 1) {   // G is a power of two
        if (j < half) red[threadIdx.x] += red[threadIdx.x + half * V];
        __syncthreads();
    }
    if (j == 0 && valid) {
        const int i = pt.off[l] + il;
        float gi;
        if (ginj) {
            gi = ginj[i];
        } else {
            gi = red[threadIdx.x];
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

// Arguments of one launch (also one run's entry of a grouped launch), the
// direct kernels, and their grouped forms (see GroupView).
struct Conv1Args {
    const float* in;
    const float* w1;
    const float* b1;
    void* out;
    uint8_t* mbits;
    int h, w;
    const DevState* st;
};
struct Wgrad1Args {
    const float* in;
    const void* dlt;
    float* part;
    int h, w;
    const DevState* st;
};
struct DecideArgs {
    const double* vpart;
    int nblk;
    long long npix;
    DevState* st;
    double* vtrace;
};
struct AccumArgs {
    const float* y;
    float* S;
    float* ybest;
    long long npix;
    const DevState* st;
};
struct AdamArgs {
    float* theta;
    float* m;
    float* v;
    float* g;
    const float* part;
    const float* ginj;
    ParamTable pt;
    float lr;
    double beta1, beta2;
    float eps;
    float* fwd;
    float* bwd;
    uint16_t* fwd16;
    uint16_t* bwd16;
    const double* lpart;
    int nloss;
    long long loss_npix;
    DevState* st;
};
static_assert(sizeof(AdamArgs) <= kArgStride && sizeof(Conv1Args) <= kArgStride, "argument table stride");
// pixels a launch processes (kernel timing)
inline long long npix_of(const Conv1Args& a) { return (long long)a.h * a.w; }
inline long long npix_of(const Wgrad1Args& a) { return (long long)a.h * a.w; }
inline long long npix_of(const DecideArgs& a) { return a.npix; }
inline long long npix_of(const AccumArgs& a) { return a.npix; }
inline long long npix_of(const AdamArgs& a) { return a.loss_npix; }

template <class A>
__device__ __forceinline__ const A& group_args(const GroupView& g, int s) {
    return *reinterpret_cast<const A*>(g.args + (size_t)s * kArgStride);
}

template <int C, bool BF>
__global__ __launch_bounds__(kBlock) void k_conv1(Conv1Args a) {
    conv1_block<C, BF>(a.in, a.w1, a.b1, a.out, a.mbits, a.h, a.w, a.st, blockIdx.x);
}
template <int C>
__global__ __launch_bounds__(kBlock) void k_conv1_group(GroupView g) {
    for_group_blocks(g, [&](int s, int vb, int) {
        const Conv1Args& a = group_args<Conv1Args>(g, s);
        conv1_block<C, true>(a.in, a.w1, a.b1, a.out, a.mbits, a.h, a.w, a.st, vb);
    });
}

template <int C, bool BF>
__global__ __launch_bounds__(kWg1Block) void k_wgrad1(Wgrad1Args a) {
    wgrad1_block<C, BF>(a.in, a.dlt, a.part, a.h, a.w, a.st, blockIdx.x, gridDim.x);
}
template <int C>
__global__ __launch_bounds__(kWg1Block) void k_wgrad1_group(GroupView g) {
    for_group_blocks(g, [&](int s, int vb, int nvb) {
        const Wgrad1Args& a = group_args<Wgrad1Args>(g, s);
        wgrad1_block<C, true>(a.in, a.dlt, a.part, a.h, a.w, a.st, vb, nvb);
    });
}

__global__ __launch_bounds__(kBlock) void k_decide(DecideArgs a) {
    decide_block(a.vpart, a.nblk, a.npix, a.st, a.vtrace);
}
__global__ __launch_bounds__(kBlock) void k_decide_group(GroupView g) {
    for_group_blocks(g, [&](int s, int, int) {
        const DecideArgs& a = group_args<DecideArgs>(g, s);
        decide_block(a.vpart, a.nblk, a.npix, a.st, a.vtrace);
    });
}

__global__ __launch_bounds__(kBlock) void k_accumulate(AccumArgs a) {
    accumulate_block(a.y, a.S, a.ybest, a.npix, a.st, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_accumulate_group(GroupView g) {
    for_group_blocks(g, [&](int s, int vb, int nvb) {
        const AccumArgs& a = group_args<AccumArgs>(g, s);
        accumulate_block(a.y, a.S, a.ybest, a.npix, a.st, vb, nvb);
    });
}

__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a) {
    adam_block(a.theta, a.m, a.v, a.g, a.part, a.ginj, a.pt, a.lr, a.beta1, a.beta2, a.eps, a.fwd, a.bwd, a.fwd16,
               a.bwd16, a.lpart, a.nloss, a.loss_npix, a.st, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(kBlock) void k_adam_group(GroupView g) {
    for_group_blocks(g, [&](int s, int vb, int nvb) {
        const AdamArgs& a = group_args<AdamArgs>(g, s);
        adam_block(a.theta, a.m, a.v, a.g, a.part, a.ginj, a.pt, a.lr, a.beta1, a.beta2, a.eps, a.fwd, a.bwd, a.fwd16,
                   a.bwd16, a.lpart, a.nloss, a.loss_npix, a.st, vb, nvb);
    });
}

// Launch one run's kernel directly, or record it for a grouped launch.
template <class K, class A>
hipError_t dispatch(K kernel, int kind, const A& a, int grid, int threads, hipStream_t s) {
    if (launch_recorder()) {
        if (kind < 0) return hipErrorNotSupported;   // no grouped form (FP32 kernels)
        return record_launch(kind, &a, sizeof(a), grid, npix_of(a), 1);
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, s, a);
    return hipGetLastError();
}


}  // namespace

hipError_t launch_minmax(const float* x, long long n, float* part, int nblk, unsigned* counter, float* lohi,
                         int* nonfinite, hipStream_t s) {
    hipLaunchKernelGGL(k_minmax, dim3(nblk), dim3(kBlock), 0, s, x, n, part, counter, lohi, nonfinite);
    return hipGetLastError();
}

hipError_t launch_prepare(const float* x, int H, int W, int C, const float* lohi, float* xs, float* ue,
                          float* uo, float* le, float* lo, int quad, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(nblocks((long long)H * W * C, kBlock)), dim3(kBlock), 0, s, x, H, W, C,
                       lohi, xs, ue, uo, le, lo, quad);
    return hipGetLastError();
}

hipError_t launch_max_project(const float* stack, int nz, long long npix, float* out, hipStream_t s) {
    const bool vec = (npix % 4) == 0 && (reinterpret_cast<uintptr_t>(stack) % 16) == 0 &&
                     (reinterpret_cast<uintptr_t>(out) % 16) == 0;
    if (vec) {
        hipLaunchKernelGGL(k_max_project<4>, dim3(nblocks(npix / 4, kBlock)), dim3(kBlock), 0, s, stack, nz, npix,
                           out);
    } else {
        hipLaunchKernelGGL(k_max_project<1>, dim3(nblocks(npix, kBlock)), dim3(kBlock), 0, s, stack, nz, npix, out);
    }
    return hipGetLastError();
}

hipError_t launch_exact_targets(const float* const* x, float* const* t, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_exact_targets, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, x[0], x[1], x[2], x[3], t[0],
                       t[1], t[2], t[3], n);
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

template <int C>
hipError_t launch_conv1_c(const float* in, const float* w1, const float* b1, void* out, uint8_t* mbits, int bf16, int h,
                    int w, const DevState* st, hipStream_t s) {
    const int grid = (int)nblocks((long long)h * w, kPxPerBlock * conv1_unroll<C>());
    const Conv1Args a{in, w1, b1, out, mbits, h, w, st};
    return bf16 ? dispatch(k_conv1<C, true>, KK_CONV1_C1 + C - 1, a, grid, kBlock, s)
                : dispatch(k_conv1<C, false>, -1, a, grid, kBlock, s);
}

hipError_t launch_conv1(const float* in, int C, const float* w1, const float* b1, void* out, uint16_t* mbits,
                        int bf16, int h, int w, const DevState* st, hipStream_t s) {
    uint8_t* mb = reinterpret_cast<uint8_t*>(mbits);
    if (C == 1) return launch_conv1_c<1>(in, w1, b1, out, mb, bf16, h, w, st, s);
    if (C == 2) return launch_conv1_c<2>(in, w1, b1, out, mb, bf16, h, w, st, s);
    return launch_conv1_c<3>(in, w1, b1, out, mb, bf16, h, w, st, s);
}

template <int C>
hipError_t launch_wgrad1_c(const float* in, const void* dlt, float* part, int nsplit, int bf16, int h, int w,
                           const DevState* st, hipStream_t s) {
    const Wgrad1Args a{in, dlt, part, h, w, st};
    return bf16 ? dispatch(k_wgrad1<C, true>, KK_WGRAD1_C1 + C - 1, a, nsplit, kWg1Block, s)
                : dispatch(k_wgrad1<C, false>, -1, a, nsplit, kWg1Block, s);
}

hipError_t launch_wgrad1(const float* in, int C, const void* dlt, float* part, int nsplit, int bf16, int h, int w,
                         const DevState* st, hipStream_t s) {
    if (C == 1) return launch_wgrad1_c<1>(in, dlt, part, nsplit, bf16, h, w, st, s);
    if (C == 2) return launch_wgrad1_c<2>(in, dlt, part, nsplit, bf16, h, w, st, s);
    return launch_wgrad1_c<3>(in, dlt, part, nsplit, bf16, h, w, st, s);
}

int head_splits(long long npix) {
    long long b = (npix + 127) / 128;
    return (int)std::max(1LL, std::min(b, (long long)kMaxHeadSplit));
}

hipError_t launch_head_train(const void* a8, const float* tgt, int C, int k, const float* w9, const float* b9,
                             void* d8, float* part, double* lpart, int nsplit, int bf16, long long npix,
                             DevState* st, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;   // grouped launches are BF16 only (fused head)
    if (bf16)
        hipLaunchKernelGGL(k_head_train<true>, dim3(nsplit), dim3(kBlock), 0, s, a8, tgt, C, k, w9, b9, d8, part,
                           lpart, npix, st);
    else
        hipLaunchKernelGGL(k_head_train<false>, dim3(nsplit), dim3(kBlock), 0, s, a8, tgt, C, k, w9, b9, d8, part,
                           lpart, npix, st);
    return hipGetLastError();
}

hipError_t launch_head_val(const void* a8, const float* xs, int C, int k, const float* w9, const float* b9,
                           float* y, double* vpart, int nblk, int bf16, long long npix, DevState* st,
                           double* vtrace, hipStream_t s) {
    if (launch_recorder()) return hipErrorNotSupported;
    if (bf16)
        hipLaunchKernelGGL(k_head_val<true>, dim3(nblk), dim3(kBlock), 0, s, a8, xs, C, k, w9, b9, y, vpart, npix,
                           (const DevState*)st);
    else
        hipLaunchKernelGGL(k_head_val<false>, dim3(nblk), dim3(kBlock), 0, s, a8, xs, C, k, w9, b9, y, vpart, npix,
                           (const DevState*)st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_decide(vpart, nblk, npix, st, vtrace, s);
}

hipError_t launch_decide(const double* vpart, int nblk, long long npix, DevState* st, double* vtrace, hipStream_t s) {
    return dispatch(k_decide, KK_DECIDE, DecideArgs{vpart, nblk, npix, st, vtrace}, 1, kBlock, s);
}

hipError_t launch_accumulate(const float* y, float* S, float* ybest, long long npix, DevState* st,
                             hipStream_t s) {
    const unsigned nb = std::min<unsigned>(nblocks(npix, kBlock * 4), 2048u);
    return dispatch(k_accumulate, KK_ACCUM, AccumArgs{y, S, ybest, npix, st}, (int)nb, kBlock, s);
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
        if (launch_recorder()) return hipErrorNotSupported;
        hipLaunchKernelGGL(k_bump_step, dim3(1), dim3(64), 0, s, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int nblk = kAdamConvBlocks + (pt.n[0] + kAdamV0 - 1) / kAdamV0 + (pt.n[kLayers] + kAdamVH - 1) / kAdamVH + 1;
    const AdamArgs a{theta, m, v, g, part, ginj, pt, lr, beta1, beta2, eps, fwd, bwd, fwd16, bwd16, lpart, nloss,
                     loss_npix, st};
    return dispatch(k_adam, ginj ? -1 : KK_ADAM, a, nblk, kBlock, s);
}

hipError_t launch_extract(const float* src, int h, int w, int C, float* out_chw, hipStream_t s) {
    const long long npix = (long long)h * w;
    hipLaunchKernelGGL(k_extract, dim3(nblocks(npix * C, kBlock)), dim3(kBlock), 0, s, src, npix, C, out_chw);
    return hipGetLastError();
}

hipError_t launch_group_misc(int kind, GroupView v, int grid, hipStream_t s) {
    switch (kind) {
        case KK_CONV1_C1: hipLaunchKernelGGL(k_conv1_group<1>, dim3(grid), dim3(kBlock), 0, s, v); break;
        case KK_CONV1_C2: hipLaunchKernelGGL(k_conv1_group<2>, dim3(grid), dim3(kBlock), 0, s, v); break;
        case KK_CONV1_C3: hipLaunchKernelGGL(k_conv1_group<3>, dim3(grid), dim3(kBlock), 0, s, v); break;
        case KK_WGRAD1_C1: hipLaunchKernelGGL(k_wgrad1_group<1>, dim3(grid), dim3(kWg1Block), 0, s, v); break;
        case KK_WGRAD1_C2: hipLaunchKernelGGL(k_wgrad1_group<2>, dim3(grid), dim3(kWg1Block), 0, s, v); break;
        case KK_WGRAD1_C3: hipLaunchKernelGGL(k_wgrad1_group<3>, dim3(grid), dim3(kWg1Block), 0, s, v); break;
        case KK_ADAM: hipLaunchKernelGGL(k_adam_group, dim3(grid), dim3(kBlock), 0, s, v); break;
        case KK_DECIDE: hipLaunchKernelGGL(k_decide_group, dim3(grid), dim3(kBlock), 0, s, v); break;
        case KK_ACCUM: hipLaunchKernelGGL(k_accumulate_group, dim3(grid), dim3(kBlock), 0, s, v); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace n2f
