// 3x3, 64->64 convolutions of the Noise2Fast network as implicit GEMMs on
// the gfx950 matrix cores (the Methods network: eight 3x3 conv+ReLU layers).
//
//   forward      out[p][co]  = relu(b[co] + sum_{t,ci} in[p+off(t)][ci] * W[t][ci][co])
//   data grad    d_in[p][ci] = [a[p][ci] > 0] * sum_{t,co} d[p+off(t)][co] * W[8-t][ci][co]
//   weight grad  dW[t][ci][co] = sum_p in[p+off(t)][ci] * d[p][co],  db[co] = sum_p d[p][co]
//
// with off(t) = (t/3 - 1, t%3 - 1) and zero padding.  The data gradient is
// the forward form with flipped taps and transposed per-tap weights, so both
// run through one kernel that takes a packed operand.
//
// Tiling (FP32 path): a 256-thread block owns a 16x16 pixel tile.  The
// 18x18x64 input halo is staged once in LDS (pixel stride 68 floats: 16-byte
// aligned rows, and 8 consecutive pixels of a 128-bit read land on 32
// distinct banks).  Each of the 4 waves computes 4 tile rows x 64 output
// channels as 4x4 MFMA 16x16x4 tiles; a lane reads 4 consecutive input
// channels with one 128-bit LDS load and feeds them to 4 MFMA steps (the K
// order inside each 16-channel chunk is permuted identically for A and B).
// B operands stream from the packed weights in L2.
#include "n2f_internal.h"

#include <algorithm>

namespace n2f {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 16;
constexpr int kHalo = kTile + 2;
constexpr int kHS = 68;  // LDS floats per staged pixel

__device__ __forceinline__ bool finished(const DevState* st) { return st != nullptr && st->done; }

// Stage the (16+2)^2 x 64 halo around tile (x0, y0) of a channels-last FP32
// activation into LDS, zero outside the image.
__device__ __forceinline__ void stage_halo_f32(float* halo, const float* __restrict__ in, int x0, int y0, int h,
                                               int w) {
    for (int idx = threadIdx.x; idx < kHalo * kHalo * 16; idx += 256) {
        const int pix = idx >> 4, q = idx & 15;
        const int hy = pix / kHalo, hx = pix - hy * kHalo;
        const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
        if (gy >= 0 && gy < h && gx >= 0 && gx < w)
            v = *reinterpret_cast<const floatx4*>(in + ((long long)gy * w + gx) * kWidth + 4 * q);
        *reinterpret_cast<floatx4*>(halo + pix * kHS + 4 * q) = v;
    }
}

// MODE 0: forward with bias + ReLU.  MODE 1: data gradient masked by [a > 0].
template <int MODE>
__global__ __launch_bounds__(256) void k_conv_f32(const float* __restrict__ in, const float* __restrict__ wpk,
                                                  const float* __restrict__ bias, const float* __restrict__ mask,
                                                  float* __restrict__ out, int h, int w, const DevState* st) {
    if (finished(st)) return;
    __shared__ __attribute__((aligned(16))) float halo[kHalo * kHalo * kHS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int x0 = blockIdx.x * kTile, y0 = blockIdx.y * kTile;
    stage_halo_f32(halo, in, x0, y0, h, w);
    __syncthreads();

    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    const floatx4* wp = reinterpret_cast<const floatx4*>(wpk);
    for (int t = 0; t < kTaps; ++t) {
        const int dy = t / 3, dx = t - 3 * (t / 3);
        const float* hrow = halo + ((4 * wv + dy) * kHalo + n + dx) * kHS + 4 * g;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            floatx4 a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = wp[(t * 16 + 4 * cc + g) * 64 + 16 * j + n];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const floatx4*>(hrow + i * kHalo * kHS + 16 * cc);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
        }
    }

    // D row (pixel x within the tile) = 4g + r, column (channel) = n.
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gy = y0 + 4 * wv + i;
        if (gy >= h) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 16 * j + n;
            float bv = 0.f;
            if (MODE == 0) bv = bias[co];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gx = x0 + 4 * g + r;
                if (gx >= w) continue;
                const long long o = ((long long)gy * w + gx) * kWidth + co;
                float v = acc[i][j][r];
                if (MODE == 0) v = fmaxf(v + bv, 0.f);
                else v = (mask[o] > 0.f) ? v : 0.f;
                out[o] = v;
            }
        }
    }
}

// Weight gradient of a 64->64 layer.  Block b accumulates tiles b, b + S,
// b + 2S, ... of 16x16 pixels and writes one partial [9*64*64 + 64].
// GEMM view: M = (t, ci) = 576 rows, N = co = 64, K = pixels; each wave owns
// 144 rows (9 M-tiles of 16) x 64 columns and takes 4 pixels per MFMA.
__global__ __launch_bounds__(256) void k_wgrad_f32(const float* __restrict__ src, const float* __restrict__ dlt,
                                                   float* __restrict__ part, int h, int w, const DevState* st) {
    if (finished(st)) return;
    __shared__ __attribute__((aligned(16))) float halo[kHalo * kHalo * kHS];
    __shared__ __attribute__((aligned(16))) float dt[kTile * kTile * kHS];
    __shared__ float dbs[4][kWidth];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int tiles_x = (w + kTile - 1) / kTile, tiles_y = (h + kTile - 1) / kTile;
    const int ntiles = tiles_x * tiles_y;

    floatx4 acc[9][4];
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dbacc = 0.f;

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int x0 = (tile % tiles_x) * kTile, y0 = (tile / tiles_x) * kTile;
        stage_halo_f32(halo, src, x0, y0, h, w);
        for (int idx = threadIdx.x; idx < kTile * kTile * 16; idx += 256) {
            const int p = idx >> 4, q = idx & 15;
            const int gy = y0 + (p >> 4), gx = x0 + (p & 15);
            floatx4 v = {0.f, 0.f, 0.f, 0.f};
            if (gy < h && gx < w) v = *reinterpret_cast<const floatx4*>(dlt + ((long long)gy * w + gx) * kWidth + 4 * q);
            *reinterpret_cast<floatx4*>(dt + p * kHS + 4 * q) = v;
        }
        __syncthreads();
        {
            const int co = threadIdx.x & 63, pg = threadIdx.x >> 6;
            float s = 0.f;
            for (int p = pg * 64; p < pg * 64 + 64; ++p) s += dt[p * kHS + co];
            dbs[pg][co] = s;
        }
        for (int kk = 0; kk < 64; ++kk) {
            const int p = 4 * kk + g;
            const int py = p >> 4, px = p & 15;
            float b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = dt[p * kHS + 16 * j + n];
#pragma unroll
            for (int ib = 0; ib < 9; ++ib) {
                const int mb = 9 * wv + ib;
                const int t = mb >> 2, ci0 = (mb & 3) * 16;
                const int dy = t / 3, dx = t - 3 * (t / 3);
                const float a = halo[((py + dy) * kHalo + px + dx) * kHS + ci0 + n];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[ib][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[j], acc[ib][j], 0, 0, 0);
            }
        }
        __syncthreads();
        if (threadIdx.x < kWidth) dbacc += ((dbs[0][threadIdx.x] + dbs[1][threadIdx.x]) + dbs[2][threadIdx.x]) + dbs[3][threadIdx.x];
    }

    float* pp = part + (long long)blockIdx.x * kConvN;
#pragma unroll
    for (int ib = 0; ib < 9; ++ib) {
        const int mb = 9 * wv + ib;
        const int t = mb >> 2, ci0 = (mb & 3) * 16;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) pp[(t * 64 + ci0 + 4 * g + r) * 64 + 16 * j + n] = acc[ib][j][r];
    }
    if (threadIdx.x < kWidth) pp[kConvW + threadIdx.x] = dbacc;
}

// ===========================================================================
// BF16 path: operands in BF16 (round to nearest even), FP32 accumulation on
// the 16x16x32 BF16 MFMA.  A lane supplies 8 consecutive K values of one row
// (A) or column (B); the MFMA sums over the 32 K values of the 4 lane groups.
// ===========================================================================
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));


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

__device__ __forceinline__ uint16_t bf16_rne(float f) { return (uint16_t)pack_bf16x2(f, 0.f); }

__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }




// MODE 0: forward, bias + ReLU.  MODE 1: data gradient masked by [a > 0].
// One persistent 512-thread block per CU.  The layer's packed weights (9 x
// 64 x 64 BF16, 72 KiB) stay in LDS for all the block's tiles.  The 8 waves
// form two groups; each group computes its own 16x16 tile from its own halo
// buffer (18 x 18 pixels x 64 BF16, the 16-byte chunks of each pixel
// XOR-swizzled by the pixel index: no padding, and the 8 lanes of a 128-bit
// read land on 32 distinct banks), so two waves share each SIMD.  While a
// group computes, the halo of its next tile is already loading into
// registers.
// The MFMA takes the weights as its first operand (rows = output channels)
// and the activations as its second (columns = pixels), so a lane's four
// accumulators are four consecutive channels of one pixel and leave as one
// 8-byte store.  The activation fragment of a tile row is read once per
// (dy, channel half): the dx = 1 and dx = 2 fragments are the same data
// moved one lane down each 16-lane DPP row, with the one pixel that enters
// at the row end taken from a broadcast LDS read.
constexpr int kHaloPix = kHalo * kHalo;               // 324 staged pixels
constexpr int kHaloChunks = kHaloPix * 8;             // 16-byte chunks per halo
constexpr int kPf = (kHaloChunks + 255) / 256;        // chunks each thread prefetches
constexpr int kDppRowShl1 = 0x101;                    // DPP control: lane n takes lane n+1 of its row
constexpr int kXHalo = kTile + 4;                     // first layer fused in: input halo side (20)
constexpr int kXHaloPix = kXHalo * kXHalo;
constexpr int kXPf = (kXHaloPix + 255) / 256;         // input values each thread prefetches

__device__ __forceinline__ int swz(int pix, int q) { return pix * 64 + ((q ^ (pix & 7)) << 3); }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// dst[n] = src[n + 1] inside each 16-lane row; the last lane of a row takes `last`.
__device__ __forceinline__ bf16x8 shift_in_row(bf16x8 src, bf16x8 last) {
    const u32x4 s = __builtin_bit_cast(u32x4, src), t = __builtin_bit_cast(u32x4, last);
    u32x4 d;
#pragma unroll
    for (int v = 0; v < 4; ++v) d[v] = (uint32_t)__builtin_amdgcn_update_dpp((int)t[v], (int)s[v], kDppRowShl1, 0xf, 0xf, false);
    return __builtin_bit_cast(bf16x8, d);
}

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
// One step of a sum over the 16 lanes of a row, toward lane 0 of the row:
// partner l + off (mod 16) for off = 8, 4 (DPP rotates), l ^ 2, l ^ 1 (quad
// permutes).  For lane 0 these are the partners of an xor butterfly.
template <int OFF>
__device__ __forceinline__ int row_step_src(int x) {
    constexpr int ctrl = OFF == 8 ? 0x128 : OFF == 4 ? 0x124 : OFF == 2 ? 0x4e : 0xb1;
    return __builtin_amdgcn_update_dpp(0, x, ctrl, 0xf, 0xf, false);
}
template <int OFF>
__device__ __forceinline__ float row_step(float x) {
    return x + __int_as_float(row_step_src<OFF>(__float_as_int(x)));
}
template <int OFF>
__device__ __forceinline__ double row_step(double x) {
    const unsigned long long u = __double_as_longlong(x);
    const unsigned long long lo = (unsigned)row_step_src<OFF>((int)(u & 0xffffffffu));
    const unsigned long long hi = (unsigned)row_step_src<OFF>((int)(u >> 32));
    return x + __longlong_as_double((long long)((hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ T row_sum16(T x) {
    return row_step<1>(row_step<2>(row_step<4>(row_step<8>(x))));
}

// BF16 bit pattern b (low 16 bits) is > 0: sign clear and not zero.
__device__ __forceinline__ bool bf16_pos(uint32_t b) { return (b & 0x8000u) == 0u && (b & 0x7fffu) != 0u; }

// The first layer (one input channel) on the 18 x 18 halo of a tile, into
// the staged BF16 halo of the layer-2 forward.  Thread gt computes 8-channel
// chunk q = gt % 8 of pixels gt / 8, gt / 8 + 32, ...: the bias plus the 9
// taps in tap order (the order of the separate first-layer kernel), ReLU,
// BF16.  Pixels outside the image stay zero (the 3x3 padding of a1).
// Interior pixels inside the image also go to global memory (a1) with their
// ReLU bit mask (the layout of the 3x3 kernels), whose two words the pixel's
// 8 lanes gather by DPP row shifts.
__device__ __forceinline__ void first_layer_halo(uint16_t* halo, const float* sxg, const float* sw1, int gt, int x0,
                                                 int y0, bool have, int h, int w, const ConvFirst& cf) {
    const int q = gt & 7;
    float wq[kTaps][8], bq[8];
#pragma unroll
    for (int t = 0; t < kTaps; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) wq[t][e] = sw1[t * kWidth + 8 * q + e];
#pragma unroll
    for (int e = 0; e < 8; ++e) bq[e] = sw1[kTaps * kWidth + 8 * q + e];
#pragma unroll
    for (int u = 0; u < kPf; ++u) {
        const int idx = gt + 256 * u;
        if (idx >= kHaloChunks) break;   // whole 8-lane pixel groups
        const int pix = idx >> 3;
        const int hy = pix / kHalo, hx = pix - hy * kHalo;
        const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
        const bool inside = have && gy >= 0 && gy < h && gx >= 0 && gx < w;
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = bq[e];
#pragma unroll
        for (int t = 0; t < kTaps; ++t) {
            const float xv = sxg[(hy + t / 3) * kXHalo + hx + t % 3];
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = fmaf(xv, wq[t][e], a[e]);
        }
        uint4 c = make_uint4(pack_bf16x2(fmaxf(a[0], 0.f), fmaxf(a[1], 0.f)), pack_bf16x2(fmaxf(a[2], 0.f), fmaxf(a[3], 0.f)),
                             pack_bf16x2(fmaxf(a[4], 0.f), fmaxf(a[5], 0.f)), pack_bf16x2(fmaxf(a[6], 0.f), fmaxf(a[7], 0.f)));
        if (!inside) c = make_uint4(0u, 0u, 0u, 0u);
        *reinterpret_cast<uint4*>(halo + swz(pix, q)) = c;
        const bool interior = inside && hy >= 1 && hy <= kTile && hx >= 1 && hx <= kTile;
        const long long gp = (long long)gy * w + gx;
        if (cf.a1 && interior)
            *reinterpret_cast<N2F_GLOBAL uint4*>(as_global(cf.a1) + gp * kWidth + 8 * q) = c;
        if (cf.m1) {
            // channel 8q + e is bit 16 (2 (q & 1) + e / 4) + 4 (q / 2) + e % 4:
            // within the low word (even q) or the high word (odd q), bit
            // 16 (e / 4) + e % 4, shifted by 4 (q / 2).  A BF16 value is > 0
            // iff its bits, as the high half of a signed 32-bit integer, are.
            const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
            uint32_t bits = 0;
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                const int e = 2 * e2;
                bits |= ((int)(cw[e2] << 16) > 0 ? 1u : 0u) << (16 * (e >> 2) + (e & 3));
                bits |= ((int)(cw[e2] & 0xffff0000u) > 0 ? 1u : 0u) << (16 * ((e + 1) >> 2) + ((e + 1) & 3));
            }
            bits <<= 4 * (q >> 1);
            // OR over the lanes of the same parity (row_shr 2, 4 stay inside
            // the pixel's aligned 8-lane group), then lane 7 takes lane 6's
            // low word (row_shr 1)
            uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0x112, 0xf, 0xf, false);
            if (q >= 2) bits |= t;
            t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0x114, 0xf, 0xf, false);
            if (q >= 4) bits |= t;
            const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)bits, 0x111, 0xf, 0xf, false);
            if (q == 7 && interior) reinterpret_cast<N2F_GLOBAL uint2*>(as_global(cf.m1))[gp] = make_uint2(lo, bits);
        }
    }
}

// ReLU bit masks of BF16 activations: 64 bits per pixel, bit 16 g + 4 j + r
// for channel 16 j + 4 g + r (g, r < 4), so each of the four lanes that hold
// a pixel's MFMA outputs owns one 16-bit word.  Bit set = the stored BF16
// value is > 0.  MODE 0 writes them (when mbits is given), MODE 1 applies
// them to the data gradient.
// MODE 2: forward of the last layer with the training head in the epilogue
// (see ConvHead); MODE 3: the same with the validation head (the output
// image and the squared error).  The lane's 16 channels of a pixel give a partial of z, the
// four lanes of the pixel add theirs by an xor butterfly, and the head
// gradient sums over a row's 16 pixels by another, then over the waves in
// order through LDS.
// Shared memory of one convolution block.  Declared in each kernel and
// passed down: declared inside the (inlined) block function, the compiler
// addressed it through extra registers and spilled.
template <int MODE>
struct ConvLds {
    static constexpr bool kHead = MODE == 2 || MODE == 3, kFirst = MODE == 4;
    __attribute__((aligned(16))) uint16_t sw[kTaps * kWidth * kWidth];
    __attribute__((aligned(16))) uint16_t hb[2][kHaloPix * kWidth];
    float shw[kHead ? kHeadN : 1];                        // head modes: head weights and bias
    float shred[kHead ? 8 : 1][kHeadN];                   // MODE 2: per-wave dW9, db9 sums
    double slred[8];                                      // head modes: per-wave BCE / squared-error sums
    float sx[2][kFirst ? kXHaloPix : 1];                  // MODE 4: input halo (20 x 20) of each group's tile
    float sw1[kFirst ? kTaps * kWidth + kWidth : 1];      // MODE 4: first-layer weights [t][co], then biases
    __attribute__((aligned(16))) float sbias[kWidth];     // forward and head modes: the layer's biases
    float stgt[2][kHead ? kTile * kTile : 1];             // head modes: each group's tile of targets
};

// Blocks [vb_lo, vb_hi) of the convolution grid of one run (nblk blocks):
// the block's own kernel runs one (vb_hi = vb_lo + 1); a block of a grouped
// launch runs consecutive blocks of one run in one pass, so the layer's
// weights are loaded once and the next block's first halo loads during the
// current block's last tile.  Block vb handles tiles 2 vb + group + 2 k nblk
// (k = 0, 1, ...) and, in the head modes, writes its own partial row, so
// what each block computes does not depend on how the blocks are run.
template <int MODE>
__device__ __forceinline__ void conv_bf16_range(const uint16_t* __restrict__ in_, const uint16_t* __restrict__ wpk_,
                                                const float* __restrict__ bias_, uint16_t* __restrict__ mbits_,
                                                uint16_t* __restrict__ out_, int h, int w, int nblk,
                                                const DevState* st, ConvHead hd, ConvFirst cf, const int vb_lo,
                                                const int vb_hi, ConvLds<MODE>& L) {
    const N2F_GLOBAL uint16_t* __restrict__ in = as_global(in_);
    const N2F_GLOBAL uint16_t* __restrict__ wpk = as_global(wpk_);
    const N2F_GLOBAL float* __restrict__ bias = as_global(bias_);
    N2F_GLOBAL uint16_t* __restrict__ mbits = as_global(mbits_);
    N2F_GLOBAL uint16_t* __restrict__ out = as_global(out_);
    auto& sw = L.sw;
    auto& hb = L.hb;
    auto& shw = L.shw;
    auto& shred = L.shred;
    auto& slred = L.slred;
    auto& sx = L.sx;
    auto& sw1 = L.sw1;
    auto& sbias = L.sbias;
    auto& stgt = L.stgt;
    constexpr bool kHead = (MODE == 2 || MODE == 3);   // head in the epilogue
    constexpr bool kFirst = (MODE == 4);               // first layer computed into the halo
    constexpr bool kFwd = (MODE == 0 || MODE == 4);    // plain forward epilogue
    // the data gradient: counted buffer loads and stores, LDS-only barriers
    // (measured: 2.7% faster; the forward measured 4% slower with them)
    constexpr bool kBufIO = (MODE == 1);
    // nblk = gridDim.x, passed among the first arguments: reading the
    // hidden grid size after the head arguments costs a second round trip
    // of scalar loads before the first global load
    // the stop flag (st is never NULL here) is read first but tested only
    // once the weight and halo loads are in flight, so its memory latency
    // hides under theirs
    const int stop = *as_global(&st->done);
    const int tid = threadIdx.x, grp = tid >> 8, gt = tid & 255;
    const int lane = tid & 63, wq = gt >> 6;
    const int g = lane >> 4, n = lane & 15;
    uint16_t* halo = hb[grp];
    // weights: all nine 16-byte loads of a thread in flight together with
    // the first halo's loads, then both go to LDS (one memory latency)
    constexpr int kWChunks = kTaps * kWidth * kWidth / 8 / 512;
    static_assert(kWChunks * 512 * 8 == kTaps * kWidth * kWidth, "weight chunks");
    uint4 wr[kWChunks];
#pragma unroll
    for (int k = 0; k < kWChunks; ++k) wr[k] = reinterpret_cast<const uint4*>(wpk)[tid + 512 * k];
    const int tiles_x = (w + kTile - 1) / kTile, tiles_y = (h + kTile - 1) / kTile;
    const int ntiles = tiles_x * tiles_y;
    const int stride = 2 * nblk;
    // tile pairs of block v (<= 0 once 2 v >= ntiles); the blocks with
    // tiles are [vb_lo, vb_work)
    auto iters_of = [&](int v) { return (ntiles - 2 * v + stride - 1) / stride; };
    const int vb_work = min(vb_hi, max(vb_lo, (ntiles + 1) / 2));

    // the halo of `tile`, zeros outside the image.  The data gradient
    // (kBufIO): buffer loads relative to the halo's top-left pixel, issued by
    // every lane (a tile past the last one reads nothing), so the compiler
    // counts them; the other modes load only the chunks inside.
    uint4 pf[kPf];
    auto fetch = [&](int tile) {
        const bool have = tile < ntiles;
        const int x0 = have ? (tile % tiles_x) * kTile : 0, y0 = have ? (tile / tiles_x) * kTile : 0;
        const auto rs = buf_rsrc(reinterpret_cast<const N2F_GLOBAL char*>(in) +
                                 ((long long)(y0 - 1) * w + (x0 - 1)) * (2 * kWidth));
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
            const int idx = gt + 256 * u;
            const int pix = idx >> 3, q = idx & 7;
            const int hy = pix / kHalo, hx = pix - hy * kHalo;
            const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
            const bool ok = have && idx < kHaloChunks && gy >= 0 && gy < h && gx >= 0 && gx < w;
            if constexpr (kBufIO) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(
                    rs, ok ? (uint32_t)((hy * w + hx) * (2 * kWidth) + 16 * q) : kBufOut, 0, 0);
                pf[u] = make_uint4(v[0], v[1], v[2], v[3]);
            } else {
                pf[u] = make_uint4(0u, 0u, 0u, 0u);
                if (ok) pf[u] = *reinterpret_cast<const uint4*>(in + ((long long)gy * w + gx) * kWidth + 8 * q);
            }
        }
    };
    // MODE 4: the input halo (tile + 2 pixels each side) of the next tile,
    // two values per thread
    float xf[kXPf];
    auto fetch_x = [&](int tile) {
        const bool have = tile < ntiles;
        const int x0 = have ? (tile % tiles_x) * kTile : 0, y0 = have ? (tile / tiles_x) * kTile : 0;
#pragma unroll
        for (int u = 0; u < kXPf; ++u) {
            const int idx = gt + 256 * u;
            const int hy = idx / kXHalo, hx = idx - hy * kXHalo;
            const int gy = y0 - 2 + hy, gx = x0 - 2 + hx;
            xf[u] = 0.f;
            if (have && idx < kXHaloPix && gy >= 0 && gy < h && gx >= 0 && gx < w)
                xf[u] = as_global(cf.x)[(long long)gy * w + gx];
        }
    };
    if (vb_lo < vb_work) {
        if constexpr (kFirst) fetch_x(2 * vb_lo + grp);
        else fetch(2 * vb_lo + grp);
    }
    float w1v[2] = {0.f, 0.f};
    if constexpr (kFirst) {
        w1v[0] = as_global(cf.w1)[tid];   // 576 weights, then 64 biases
        if (tid < kTaps * kWidth + kWidth - 512)
            w1v[1] = (tid + 512 < kTaps * kWidth) ? as_global(cf.w1)[tid + 512]
                                                  : as_global(cf.b1)[tid + 512 - kTaps * kWidth];
    }
    const float hwv = (kHead && tid < kHeadN) ? as_global(hd.w9)[tid] : 0.f;
    const float bvv = (MODE != 1 && tid < kWidth) ? bias[tid] : 0.f;
    asm volatile("" ::: "memory");   // keeps those loads ahead of the test
    if (stop) return;
    if (MODE != 1 && tid < kWidth) sbias[tid] = bvv;
    if constexpr (kFirst) {
        sw1[tid] = w1v[0];
        if (tid < kTaps * kWidth + kWidth - 512) sw1[tid + 512] = w1v[1];
    }
    if (kHead) {
        if (tid < kHeadN) shw[tid] = hwv;
        for (int i = tid; i < 8 * kHeadN; i += 512) (&shred[0][0])[i] = 0.f;
        if (tid < 8) slred[tid] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < kWChunks; ++k) reinterpret_cast<uint4*>(sw)[tid + 512 * k] = wr[k];

    // head modes: block v's partial row from the per-wave sums (waves in
    // order), then the sums start again from zero; called after a barrier
    auto flush = [&](int v) {
        if (MODE == 2 && tid < kHeadN) {
            float sum = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q) sum += shred[q][tid];
            as_global(hd.part)[(long long)v * kHeadN + tid] = sum;
        }
        if (tid == 0) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) sum += slred[q];
            as_global(hd.lpart)[v] = sum;
            // one Adam step follows this head: count it (no other block reads t)
            if (MODE == 2 && v == 0) *as_global(&hd.st->t) += 1;
        }
        __syncthreads();
        if (MODE == 2)
            for (int i = tid; i < 8 * kHeadN; i += 512) (&shred[0][0])[i] = 0.f;
        if (tid < 8) slred[tid] = 0.0;
    };
    // the work is the sequence of (block vb, tile k) pairs, k < iters_of(vb)
    int vb = vb_lo, k = 0, iters = iters_of(vb_lo);
    while (vb < vb_work) {
        const int tile = 2 * vb + grp + k * stride;
        const bool have = tile < ntiles;
        const int x0 = have ? (tile % tiles_x) * kTile : 0, y0 = have ? (tile / tiles_x) * kTile : 0;
        int nvb = vb, nk = k + 1;   // the next pair
        if (nk >= iters) {
            nvb = vb + 1;
            nk = 0;
        }
        const bool more = nvb < vb_work;
        const int ntile = 2 * nvb + grp + nk * stride;
        // kBufIO: the barriers of the tile loop wait for LDS traffic only, so
        // the next tile's loads stay in flight across them; the mask words
        // (data gradient) load before the next tile's halo, since loads
        // complete in order and waiting for them then leaves the halo in
        // flight
        const int ftile = more ? ntile : ntiles;   // past the last tile: reads nothing
        uint32_t mk[4];
        if constexpr (MODE == 1) {
            const auto rm = buf_rsrc(mbits + ((long long)y0 * w + x0) * 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gy = y0 + 4 * wq + i, gx = x0 + n;
                const bool ok = have && gy < h && gx < w;
                mk[i] = __builtin_amdgcn_raw_buffer_load_b16(
                    rm, ok ? (uint32_t)((((4 * wq + i) * w + n) * 4 + g) * 2) : kBufOut, 0, 0);
            }
        }
        if constexpr (kFirst) {
#pragma unroll
            for (int u = 0; u < kXPf; ++u) {
                const int idx = gt + 256 * u;
                if (idx < kXHaloPix) sx[grp][idx] = xf[u];
            }
            __syncthreads();
            if (more) fetch_x(ntile);   // in flight during the rest of the tile
            first_layer_halo(halo, sx[grp], sw1, gt, x0, y0, have, h, w, cf);
            __syncthreads();
        } else {
#pragma unroll
            for (int u = 0; u < kPf; ++u) {
                const int idx = gt + 256 * u;
                if (idx < kHaloChunks) *reinterpret_cast<uint4*>(halo + swz(idx >> 3, idx & 7)) = pf[u];
            }
            if constexpr (kBufIO) {
                lds_barrier();
                fetch(ftile);   // in flight during the MFMA loop
            } else {
                __syncthreads();
                if (more) fetch(ntile);   // in flight during the MFMA loop
            }
        }

        // head modes: target pixel gt of the tile, loaded before the MFMA loop
        // and staged in LDS after it
        float tq = 0.f;
        if (kHead) {
            const int gy = y0 + (gt >> 4), gx = x0 + (gt & 15);
            if (have && gy < h && gx < w) tq = as_global(hd.tgt)[((long long)gy * w + gx) * hd.C + hd.k];
        }
        floatx4 acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                // activation fragments of tile rows 4wq+i at dx = 0 (lane n: pixel n),
                // and the pixels 16, 17 that enter at the row end for dx = 1, 2
                // (broadcast reads: an exec-masked read for the last lane alone
                // splits the unrolled MFMA block into basic blocks and measured slower)
                bf16x8 a0[4], e1[4], e2[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int prow = (4 * wq + i + dy) * kHalo;
                    a0[i] = *reinterpret_cast<const bf16x8*>(halo + swz(prow + n, 4 * kc + g));
                    e1[i] = *reinterpret_cast<const bf16x8*>(halo + swz(prow + 16, 4 * kc + g));
                    e2[i] = *reinterpret_cast<const bf16x8*>(halo + swz(prow + 17, 4 * kc + g));
                }
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    if (dx > 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) a0[i] = shift_in_row(a0[i], dx == 1 ? e1[i] : e2[i]);
                    }
                    // B fragment of tap t, channels 8(4kc+g).. of output column 16j+n
                    const int it = 2 * (3 * dy + dx) + kc;
                    bf16x8 wb[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        wb[j] = *reinterpret_cast<const bf16x8*>(sw + ((4 * it + g) * 64 + 16 * j + n) * 8);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[j], a0[i], acc[i][j], 0, 0, 0);
                }
            }
        }

        if (kHead) {
            stgt[grp][gt] = tq;
            __syncthreads();
        }
        // D row = channel 16j + 4g + r, column = pixel x = n of tile row 4wq + i.
        if (kHead && have) {
            const int gx = x0 + n;
            float hg[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) hg[j][r] = 0.f;
            float hbs = 0.f;
            double hls = 0.0;
            // the biases are read from LDS where they are used (16-byte words):
            // held in registers across the pixel loop they push the grouped
            // kernel past 256 VGPRs
            const float hb9 = shw[kWidth];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gy = y0 + 4 * wq + i;
                const bool valid = gy < h && gx < w;
                const long long pix = (long long)gy * w + gx;
                const float t = stgt[grp][(4 * wq + i) * kTile + n];   // 0 outside the image
                // a8 as the BF16 value the forward would store, channels
                // 16 j + 4 g .. + 3 of this lane: computed where used (twice:
                // for z, then for the delta and dW9) rather than held, to
                // keep the grouped kernel within 256 VGPRs
                auto a_of = [&](int j, float (&av)[4]) __attribute__((always_inline)) {
                    const float4 b4 = *reinterpret_cast<const float4*>(&sbias[16 * j + 4 * g]);
                    const float bv[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                    for (int r = 0; r < 4; r += 2) {
                        const uint32_t pk = pack_bf16x2(fmaxf(acc[i][j][r] + bv[r], 0.f),
                                                        fmaxf(acc[i][j][r + 1] + bv[r + 1], 0.f));
                        av[r] = __uint_as_float(pk << 16);
                        av[r + 1] = __uint_as_float(pk & 0xffff0000u);
                    }
                };
                float zp = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float av[4];
                    a_of(j, av);
#pragma unroll
                    for (int r = 0; r < 4; ++r) zp = fmaf(av[r], shw[16 * j + 4 * g + r], zp);
                }
                zp = add_xor32(add_xor16(zp));
                const float z = zp + hb9;
                const float y = 1.0f / (1.0f + expf(-z));
                if (MODE == 3) {
                    // validation: the output pixel and its squared error against the noisy image
                    if (valid && g == 0) {
                        as_global(hd.y)[pix] = y;
                        const double e = (double)y - (double)t;
                        hls += e * e;
                    }
                    continue;
                }
                const float d = valid ? (y - t) * hd.invP : 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float av[4];
                    a_of(j, av);
                    if (valid) {
                        float dv[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) dv[r] = av[r] > 0.f ? d * shw[16 * j + 4 * g + r] : 0.f;
                        const uint2 o = make_uint2(pack_bf16x2(dv[0], dv[1]), pack_bf16x2(dv[2], dv[3]));
                        *reinterpret_cast<uint2*>(out + pix * kWidth + 16 * j + 4 * g) = o;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) hg[j][r] = fmaf(d, av[r], hg[j][r]);
                }
                if (valid && g == 0) {
                    hbs += d;
                    hls += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - t * z);
                }
            }
            // the 16 pixels (lanes n) of each row, then the wave's slot
            if (MODE == 2) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) hg[j][r] = row_sum16(hg[j][r]);
                hbs = row_sum16(hbs);
            }
            hls = row_sum16(hls);
            if (n == 0) {
                const int wv = tid >> 6;
                if (MODE == 2) {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) shred[wv][16 * j + 4 * g + r] += hg[j][r];
                }
                if (g == 0) {
                    if (MODE == 2) shred[wv][kWidth] += hbs;
                    slred[wv] += hls;
                }
            }
        }
        if constexpr (kBufIO) {
            // buffer writes relative to pixel (y0, x0): those outside the
            // image (or of a tile past the last) are dropped
            float bv[4][4];
            if (kFwd) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) bv[j][r] = sbias[16 * j + 4 * g + r];
            }
            const int gx = x0 + n;
            const bool want_mask = kFwd && mbits != nullptr;   // the forward's mask words (not in validation)
            const long long t0 = (long long)y0 * w + x0;
            const auto ro = buf_rsrc(out + t0 * kWidth);
            const auto rmk = buf_rsrc(mbits + t0 * 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gy = y0 + 4 * wq + i;
                const bool ok = have && gy < h && gx < w;
                const int rel = (4 * wq + i) * w + n;   // pixel relative to (y0, x0)
                uint32_t word = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = kFwd ? fmaxf(acc[i][j][r] + bv[j][r], 0.f) : acc[i][j][r];
                    uint2 o = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                    if (MODE == 1) {
                        const uint32_t m = mk[i] >> (4 * j);
                        o.x &= ((m & 1u) ? 0x0000ffffu : 0u) | ((m & 2u) ? 0xffff0000u : 0u);
                        o.y &= ((m & 4u) ? 0x0000ffffu : 0u) | ((m & 8u) ? 0xffff0000u : 0u);
                    } else if (want_mask) {
                        // a BF16 value is > 0 iff its bits, as the high half of
                        // a signed 32-bit integer, are > 0 (-0 is not)
                        word |= ((int)(o.x << 16) > 0 ? 1u : 0u) << (4 * j);
                        word |= ((int)(o.x & 0xffff0000u) > 0 ? 2u : 0u) << (4 * j);
                        word |= ((int)(o.y << 16) > 0 ? 4u : 0u) << (4 * j);
                        word |= ((int)(o.y & 0xffff0000u) > 0 ? 8u : 0u) << (4 * j);
                    }
                    __builtin_amdgcn_raw_buffer_store_b64((__attribute__((ext_vector_type(2))) unsigned int){o.x, o.y},
                                                          ro, ok ? (uint32_t)((rel * kWidth + 4 * g + 16 * j) * 2)
                                                                 : kBufOut,
                                                          0, 0);
                }
                if (kFwd)
                    __builtin_amdgcn_raw_buffer_store_b16(
                        (unsigned short)word, rmk, ok && want_mask ? (uint32_t)((rel * 4 + g) * 2) : kBufOut, 0, 0);
            }
        } else if (!kHead && have) {
            float bv[4][4];
            if (kFwd) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) bv[j][r] = sbias[16 * j + 4 * g + r];
            }
            const int gx = x0 + n;
            const bool want_mask = kFwd && mbits != nullptr;   // the forward's mask words (not in validation)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gy = y0 + 4 * wq + i;
                if (gy >= h || gx >= w) continue;
                const long long base = ((long long)gy * w + gx) * kWidth + 4 * g;
                uint32_t word = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] = kFwd ? fmaxf(acc[i][j][r] + bv[j][r], 0.f) : acc[i][j][r];
                    uint2 o = make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
                    if (want_mask) {
                        word |= ((int)(o.x << 16) > 0 ? 1u : 0u) << (4 * j);
                        word |= ((int)(o.x & 0xffff0000u) > 0 ? 2u : 0u) << (4 * j);
                        word |= ((int)(o.y << 16) > 0 ? 4u : 0u) << (4 * j);
                        word |= ((int)(o.y & 0xffff0000u) > 0 ? 8u : 0u) << (4 * j);
                    }
                    *reinterpret_cast<uint2*>(out + base + 16 * j) = o;
                }
                if (want_mask) mbits[((long long)gy * w + gx) * 4 + g] = (uint16_t)word;
            }
        }
        // the next tile's halo overwrites this buffer
        if constexpr (kBufIO) lds_barrier();
        else __syncthreads();
        if (kHead && nk == 0) flush(vb);   // block vb is complete
        vb = nvb;
        k = nk;
        if (k == 0) iters = iters_of(vb);
    }
    // blocks without tiles still write their (zero) partial rows
    if (kHead) {
        for (int v = max(vb_lo, vb_work); v < vb_hi; ++v) {
            __syncthreads();
            flush(v);
        }
    }
}

// Arguments of one launch of k_conv_bf16 (also one run's entry of a grouped
// launch).
struct ConvArgs {
    const uint16_t* in;
    const uint16_t* wpk;
    const float* bias;
    uint16_t* mbits;
    uint16_t* out;
    int h, w, nblk;
    const DevState* st;
    ConvHead hd;
    ConvFirst cf;
};
static_assert(sizeof(ConvArgs) <= kArgStride, "argument table stride");
inline long long npix_of(const ConvArgs& a) { return (long long)a.h * a.w; }

// Separate parameters (not one argument struct): the struct form costs
// registers here, and this kernel has none to spare.
template <int MODE>
__global__ __launch_bounds__(512) void k_conv_bf16(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wpk,
                                                   const float* __restrict__ bias, uint16_t* __restrict__ mbits,
                                                   uint16_t* __restrict__ out, int h, int w, int nblk,
                                                   const DevState* st, ConvHead hd, ConvFirst cf) {
    __shared__ ConvLds<MODE> L;
    conv_bf16_range<MODE>(in, wpk, bias, mbits, out, h, w, nblk, st, hd, cf, blockIdx.x, blockIdx.x + 1, L);
}

// The same convolution over a group of runs (see GroupView): block b runs
// the consecutive virtual blocks [starts[b], starts[b + 1]) (balanced by
// their tiles on the host), one run's share at a time.
template <int MODE>
__global__ __launch_bounds__(512) void k_conv_bf16_group(GroupView g) {
    __shared__ ConvLds<MODE> L;
    const int n = g.prefix[0];
    const int* pre = g.prefix + 1;
    const int lo = g.starts[blockIdx.x], hi = g.starts[blockIdx.x + 1];
    int s = 0;
    for (int gv = lo; gv < hi;) {
        while (s < n && gv >= pre[s + 1]) ++s;
        const int end = min(hi, pre[s + 1]);
        __syncthreads();   // shared memory of the previous run's blocks is free
        const ConvArgs a = load_uniform(reinterpret_cast<const ConvArgs*>(g.args + (size_t)s * kArgStride));
        conv_bf16_range<MODE>(a.in, a.wpk, a.bias, a.mbits, a.out, a.h, a.w, a.nblk, a.st, a.hd, a.cf, gv - pre[s],
                              end - pre[s], L);
        gv = end;
    }
}

// Grid of the BF16 convolution: one block (two tiles in flight) per CU at most.
int conv_bf16_blocks(int h, int w) {
    const int tiles = ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
    const int b = (tiles + 1) / 2;
    return b < 256 ? b : 256;
}

// BF16 weight gradient of a 64->64 layer.  GEMM view as in the FP32 kernel
// (M = (t, ci) = 576, N = co = 64, K = pixels).  The grid is 4 x nsplit
// blocks: block (s, q) owns the 144 rows of input-channel quarter q (9 taps
// x 16 channels) over the tiles s, s + nsplit, s + 2 nsplit, ...; so the
// partial of split s is written by four blocks, each its own rows, and a
// layer has only nsplit partials to reduce.  The four quarter blocks of a
// split are placed on one XCD (block ids 8 apart), where they share the
// delta tiles through that XCD's L2.
//
// Per tile, wave (pr, oh) of the 8 takes the 64 pixels 64 pr .. (four tile
// rows, two K steps) for the 18 output tiles of its half oh of co (9 taps
// x 2 blocks of 16).  Both operands stay pixel-major in LDS and are read
// with the gfx950 16-bit transpose load: within a group of 16 lanes,
// row-lane r addresses pixel p0 + r/4 and channels c0 + 4(r%4).., and lane
// L then holds channel c0 + L of pixels p0..p0+3; two such loads give the 8
// K values of an MFMA fragment.  A tap shift is only a different row
// address.
//
// Tiles go from global memory straight into LDS (16-byte buffer loads that
// write LDS), three buffers deep: while tile it is multiplied, tile it + 1
// may still be landing and tile it + 2 is requested.  A wave's load
// instruction fills 64 consecutive 16-byte LDS slots, one per lane, so
// each lane fetches the chunk that the (bank-spreading) layout puts in its
// slot; chunks outside the image come back as zeros (out-of-range buffer
// offsets read zero).  Each thread issues the same six loads per tile, so
// a wave waits only for the loads two tiles old, and the barriers wait for
// LDS traffic only.  The bias gradient is summed from the staged delta with
// 16-byte reads, a quarter of it in each quarter block.  At the end the
// waves' sums are added in wave order through LDS, three taps at a time.
constexpr int kWgPSA = 16;                                 // bf16 per staged halo pixel (one quarter)
constexpr int kWgPSB = 64;                                 // bf16 per staged delta pixel (chunks XOR-placed)
constexpr int kWgHaloSlots = 704;                          // 16-byte slots of the halo quarter (648 used): 11 x 64
constexpr int kWgSlots = 3072;                             // slots per buffer: halo, delta (2048), unused rest
constexpr int kWgDma = kWgSlots / 512;                     // loads per thread per tile
constexpr int kWgHaloE = kWgHaloSlots * 8;                 // bf16 offset of the delta in a buffer
constexpr int kWgBufE = kWgSlots * 8;                      // bf16 per buffer (48 KB)
constexpr int kWgRedT = 3;                                 // taps per pass of the final reduction
static_assert(kWgHaloSlots >= kHalo * kHalo * 2 && kWgHaloSlots % 64 == 0, "halo slots");
static_assert(kWgHaloSlots + kTile * kTile * 8 <= kWgSlots && kWgSlots % 512 == 0, "buffer slots");
static_assert(8 * 2 * kWgRedT * 64 * 16 <= kWgBufE * 2, "one pass of the reduction fits a buffer");
static_assert((256 + 32) * 16 * 4 <= kWgBufE * 2, "the bias sums fit a buffer");

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;

__device__ __forceinline__ bf16x8 tr16_frag(const uint16_t* p0, const uint16_t* p1) {
    const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
        (lds_bf16x4*)((__attribute__((address_space(3))) uint16_t*)p0));
    const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
        (lds_bf16x4*)((__attribute__((address_space(3))) uint16_t*)p1));
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// LDS placement of the staged operands, so that the transpose reads of the
// lane groups LDS serves together hit distinct banks: halo pixel (hy, hx)
// sits in 32-byte slot hy * 18 + wg_hslot(hx) (columns 8..15 swap their
// halves, so the columns x and x + 8 that two lane groups read together
// never share a bank, and a row shift stays a constant offset); delta
// pixel p keeps its 128-byte row and its 16-byte chunk c moves to
// c ^ wg_dswz(p).  Both maps are their own inverses.
__device__ __forceinline__ int wg_hslot(int hx) { return hx ^ (((hx >> 3) & 1) << 2); }
__device__ __forceinline__ int wg_dswz(int p) { return (p & 2) | ((p >> 1) & 4); }
__device__ __forceinline__ int wg_dt(int p, int ch) { return p * kWgPSB + ((((ch >> 3) ^ wg_dswz(p))) << 3) + (ch & 7); }

// A thread's load k of every tile fills LDS slot 64 (wv + 8k) + lane; the
// first 11 such groups of 64 slots are the halo quarter's (channels
// 16q..16q+15 of the 18x18 pixels around the tile), the next 32 the 16x16x64
// delta tile's.  Which chunk a slot holds is the same for every tile, so it
// is worked out once per block: `rel`, the chunk's byte offset from its base
// pixel (the halo's top-left (y0 - 1, x0 - 1) or the tile's (y0, x0)), or
// kBufOut for the slots past the operands; `rc`, the pixel's row and column
// relative to (y0 - 1, x0 - 1), in bits 0-7 and 8-15.
struct WgSlots {
    uint32_t rel[kWgDma];
    uint32_t rc[kWgDma];
};
__device__ __forceinline__ WgSlots wg_slots(int q, int w) {
    WgSlots sl;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < kWgDma; ++k) {
        const int grp = wv + 8 * k;   // wave-uniform
        const int s = 64 * grp + lane;
        if (grp < kWgHaloSlots / 64) {
            // halo slot s: pixel slot s / 2 = hy * 18 + wg_hslot(hx), half s % 2
            const int ps = s >> 1, hy = ps / kHalo, hx = wg_hslot(ps - hy * kHalo);
            sl.rel[k] = s < kHalo * kHalo * 2 ? (uint32_t)((hy * w + hx) * (2 * kWidth) + 2 * (16 * q + 8 * (s & 1)))
                                              : kBufOut;
            sl.rc[k] = (uint32_t)(hy | (hx << 8));
        } else {
            // delta slot: pixel p = d / 8, chunk (d % 8) ^ wg_dswz(p)
            const int d = s - kWgHaloSlots;
            const int p = d >> 3, cq = (d & 7) ^ wg_dswz(p);
            const int py = p >> 4, px = p & 15;
            sl.rel[k] = d < kTile * kTile * 8 ? (uint32_t)((py * w + px) * (2 * kWidth) + 16 * cq) : kBufOut;
            sl.rc[k] = (uint32_t)((py + 1) | ((px + 1) << 8));
        }
    }
    return sl;
}

// Request tile (x0, y0) into the LDS buffer `buf`: the slots whose pixel
// lies outside the image (or past the operands) read zeros.
__device__ __forceinline__ void wg_request(uint16_t* buf, const WgSlots& sl, const N2F_GLOBAL uint16_t* src,
                                           const N2F_GLOBAL uint16_t* dlt, int x0, int y0, int h, int w) {
    typedef __attribute__((address_space(3))) void lds_void;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // byte bases: the halo's top-left pixel (y0 - 1, x0 - 1) and the tile's (y0, x0)
    const long long hb = ((long long)(y0 - 1) * w + (x0 - 1)) * (2 * kWidth);
    const long long db = ((long long)y0 * w + x0) * (2 * kWidth);
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(reinterpret_cast<const N2F_GLOBAL char*>(src) + hb);
    const __amdgpu_buffer_rsrc_t rd = buf_rsrc(reinterpret_cast<const N2F_GLOBAL char*>(dlt) + db);
#pragma unroll
    for (int k = 0; k < kWgDma; ++k) {
        const int grp = wv + 8 * k;   // wave-uniform
        const uint32_t gy = (uint32_t)(y0 - 1 + (int)(sl.rc[k] & 0xffu));
        const uint32_t gx = (uint32_t)(x0 - 1 + (int)((sl.rc[k] >> 8) & 0xffu));
        const uint32_t off = (gy < (uint32_t)h && gx < (uint32_t)w) ? sl.rel[k] : kBufOut;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(grp < kWgHaloSlots / 64 ? rh : rd, (lds_void*)(buf + 512 * grp), 16,
                                                 off, 0, 0, 0);
    }
}

// One block of the weight-gradient grid: block `b` of `nb` = 4 x nsplit.
__device__ __forceinline__ void wgrad_bf16_block(const uint16_t* __restrict__ src_, const uint16_t* __restrict__ dlt_,
                                                 float* __restrict__ part, int h, int w, const DevState* st,
                                                 const int b, const int nb) {
    const N2F_GLOBAL uint16_t* src = as_global(src_);
    const N2F_GLOBAL uint16_t* dlt = as_global(dlt_);
    const int stop = *as_global(&st->done);   // tested once the first tiles' loads are in flight
    // three tile buffers, separate objects so that the compiler tracks the
    // loads into each one apart
    __shared__ __attribute__((aligned(16))) uint16_t buf0[kWgBufE];
    __shared__ __attribute__((aligned(16))) uint16_t buf1[kWgBufE];
    __shared__ __attribute__((aligned(16))) uint16_t buf2[kWgBufE];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, r = lane & 15;
    // wave wv: pixels 64 (wv / 2) .. + 63 of each tile (two K steps) and
    // output-channel blocks 2 (wv % 2), 2 (wv % 2) + 1
    const int pr = wv >> 1, oh = wv & 1;
    const int nsplit = nb / 4;
    int sp, q;
    if ((nsplit & 7) == 0) {
        q = (b >> 3) & 3;
        sp = (b & 7) + 8 * (b >> 5);
    } else {
        q = b / nsplit;
        sp = b - q * nsplit;
    }
    const int tiles_x = (w + kTile - 1) / kTile, tiles_y = (h + kTile - 1) / kTile;
    const int ntiles = tiles_x * tiles_y;
    const int nmine = sp < ntiles ? (ntiles - sp + nsplit - 1) / nsplit : 0;

    floatx4 acc[9][2];
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // bias gradient of the block's 16 channels 16 q ..: thread = (pixel
    // tid / 2 of each tile, 8-channel chunk 2 q + tid % 2); every quarter
    // block does a quarter of the work
    float db[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    // the requests past the block's last tile repeat that tile, so that
    // every step issues the same loads and the waits stay exact
    const WgSlots slots = wg_slots(q, w);
    auto request = [&](uint16_t* buf, int it) __attribute__((always_inline)) {
        const int tile = sp + min(it, nmine - 1) * nsplit;
        wg_request(buf, slots, src, dlt, (tile % tiles_x) * kTile, (tile / tiles_x) * kTile, h, w);
    };
    if (nmine > 0) {
        request(buf0, 0);
        request(buf1, 1);
    }
    if (stop) {
        wait_vmcnt<0>();   // the LDS the loads write stays allocated until they land
        return;
    }
    const int rp = r >> 2, rc = 4 * (r & 3);

    // tile `it` is in `cur` (loaded two steps ago); `nxt` held tile it - 1.
    // The steps past the last tile (up to two, rounding the loop to whole
    // buffer cycles) still wait, synchronise and request, so that every
    // path issues the same loads, and only skip the multiply.
    auto step = [&](const uint16_t* cur, uint16_t* nxt, int it) __attribute__((always_inline)) {
        wait_vmcnt<kWgDma>();   // this wave's loads of tile it have landed (tile it + 1's may not)
        lds_barrier();          // every wave's have, and every wave is done with tile it - 1
        request(nxt, it + 2);
        if (it >= nmine) return;
        const uint16_t* halo = cur;
        const uint16_t* dt = cur + kWgHaloE;
        {
            const uint4 v = *reinterpret_cast<const uint4*>(dt + wg_dt(tid >> 1, 8 * (2 * q + (tid & 1))));
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                db[2 * e] += __uint_as_float(u[e] << 16);
                db[2 * e + 1] += __uint_as_float(u[e] & 0xffff0000u);
            }
        }
        // K step 1 covers the two pixel rows below K step 0, so its dy = 0
        // fragments are K step 0's dy = 2 fragments: read once, used twice
        bf16x8 a_dy2[3];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            // pixels of K step ks: k0 = 64 pr + 32 ks + 8 g + r/4 and k0 + 4
            const int k0 = 64 * pr + 32 * ks + 8 * g + rp, k1 = k0 + 4;
            const int py0 = k0 >> 4, px0 = k0 & 15, py1 = k1 >> 4, px1 = k1 & 15;
            bf16x8 bfr[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int cb = 16 * (2 * oh + j) + rc;
                bfr[j] = tr16_frag(dt + wg_dt(k0, cb), dt + wg_dt(k1, cb));
            }
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int dy = t / 3, dx = t - 3 * (t / 3);
                const bf16x8 a = (ks == 1 && dy == 0)
                                     ? a_dy2[dx]
                                     : tr16_frag(halo + ((py0 + dy) * kHalo + wg_hslot(px0 + dx)) * kWgPSA + rc,
                                                 halo + ((py1 + dy) * kHalo + wg_hslot(px1 + dx)) * kWgPSA + rc);
                if (ks == 0 && dy == 2) a_dy2[dx] = a;
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[j], acc[t][j], 0, 0, 0);
            }
        }
    };
    for (int it = 0; it < nmine; it += 3) {
        step(buf0, buf2, it);
        step(buf1, buf0, it + 1);
        step(buf2, buf1, it + 2);
    }
    wait_vmcnt<0>();   // the requests past the last tile
    lds_barrier();     // every wave is done with the tiles: the buffers are free

    // sum the 4 waves of each channel half in order, three taps per pass: a
    // lane's 4 accumulator values (rows 4 (lane / 16) + e, column lane % 16
    // of an MFMA tile) move as one 16-byte LDS word; a reader adds the same
    // word of the 4 waves and stores its 4 rows
    float4* red = reinterpret_cast<float4*>(buf0);
    N2F_GLOBAL float* pp = as_global(part) + (long long)sp * kConvN;
#pragma unroll
    for (int pass = 0; pass < kTaps / kWgRedT; ++pass) {
        const int t0 = pass * kWgRedT;
#pragma unroll
        for (int tt = 0; tt < kWgRedT; ++tt)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const floatx4 v = acc[t0 + tt][j];
                red[(wv * 2 * kWgRedT + tt * 2 + j) * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
            }
        lds_barrier();
        for (int gi = tid; gi < kWgRedT * 2 * 2 * 64; gi += 512) {
            const int ln = gi & 63, jj = (gi >> 6) & 1, ohh = (gi >> 7) & 1, tt = gi >> 8;
            float4 sum = red[(ohh * 2 * kWgRedT + tt * 2 + jj) * 64 + ln];
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                const float4 x = red[((2 * k + ohh) * 2 * kWgRedT + tt * 2 + jj) * 64 + ln];
                sum.x += x.x;
                sum.y += x.y;
                sum.z += x.z;
                sum.w += x.w;
            }
            const int co = 16 * (2 * ohh + jj) + (ln & 15), cil = 4 * (ln >> 4);
            N2F_GLOBAL float* o = pp + ((t0 + tt) * kWidth + 16 * q + cil) * kWidth + co;
            o[0] = sum.x;
            o[kWidth] = sum.y;
            o[2 * kWidth] = sum.z;
            o[3 * kWidth] = sum.w;
        }
        lds_barrier();
    }
    // the 256 pixel slots of each channel: 32 runs of 8 slots, then the runs,
    // in order (per-thread sums of the block's 16 channels, in a tile buffer)
    float (*dbs)[16] = reinterpret_cast<float (*)[16]>(buf1);
    float (*dbs2)[16] = dbs + 256;
#pragma unroll
    for (int e = 0; e < 8; ++e) dbs[tid >> 1][8 * (tid & 1) + e] = db[e];
    lds_barrier();
    {
        const int c = tid & 15, run = tid >> 4;
        float sum = dbs[8 * run][c];
#pragma unroll
        for (int k = 1; k < 8; ++k) sum += dbs[8 * run + k][c];
        dbs2[run][c] = sum;
    }
    lds_barrier();
    if (tid < 16) {
        float sum = dbs2[0][tid];
#pragma unroll
        for (int k = 1; k < 32; ++k) sum += dbs2[k][tid];
        pp[kConvW + 16 * q + tid] = sum;
    }
}

struct WgradArgs {
    const uint16_t* src;
    const uint16_t* dlt;
    float* part;
    int h, w;
    const DevState* st;
};

__global__ __launch_bounds__(512) void k_wgrad_bf16(WgradArgs a) {
    wgrad_bf16_block(a.src, a.dlt, a.part, a.h, a.w, a.st, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(512) void k_wgrad_bf16_group(GroupView g) {
    for_group_blocks(g, [&](int s, int vb, int nvb) {
        const WgradArgs a = load_uniform(reinterpret_cast<const WgradArgs*>(g.args + (size_t)s * kArgStride));
        wgrad_bf16_block(a.src, a.dlt, a.part, a.h, a.w, a.st, vb, nvb);
    });
}

// Launch one run's kernel directly, or record it for a grouped launch.
template <int MODE>
hipError_t dispatch_conv(const ConvArgs& a, int grid, hipStream_t s) {
    constexpr int kind = MODE == 0 ? KK_CONV_FWD : MODE == 1 ? KK_CONV_DGRAD : MODE == 2 ? KK_CONV_HEAD
                                   : MODE == 3 ? KK_CONV_VAL : KK_CONV_FIRST;
    if (launch_recorder()) {
        // cost of one virtual block: the tile pairs it runs (at least one)
        const int ntiles = ((a.w + kTile - 1) / kTile) * ((a.h + kTile - 1) / kTile);
        const int cost = std::max(1, (ntiles + 2 * a.nblk - 1) / (2 * a.nblk));
        return record_launch(kind, &a, sizeof(a), grid, npix_of(a), cost);
    }
    hipLaunchKernelGGL(k_conv_bf16<MODE>, dim3(grid), dim3(512), 0, s, a.in, a.wpk, a.bias, a.mbits, a.out, a.h, a.w,
                       a.nblk, a.st, a.hd, a.cf);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_conv_fwd(const void* in, const void* wpk, const float* bias, void* out, uint16_t* mbits, int bf16,
                           int h, int w, const DevState* st, hipStream_t s) {
    dim3 grid((w + kTile - 1) / kTile, (h + kTile - 1) / kTile);
    if (bf16) {
        const int nb = conv_bf16_blocks(h, w);
        return dispatch_conv<0>(ConvArgs{(const uint16_t*)in, (const uint16_t*)wpk, bias, mbits, (uint16_t*)out, h, w,
                                         nb, st, ConvHead{}, ConvFirst{}},
                                nb, s);
    }
    if (launch_recorder()) return hipErrorNotSupported;   // grouped launches are BF16 only
    hipLaunchKernelGGL(k_conv_f32<0>, grid, dim3(256), 0, s, (const float*)in, (const float*)wpk, bias,
                       (const float*)nullptr, (float*)out, h, w, st);
    return hipGetLastError();
}

hipError_t launch_conv_fwd_head(const void* in, const void* wpk, const float* bias, void* d8, const ConvHead& hd,
                                int nblk, int h, int w, const DevState* st, hipStream_t s) {
    if (nblk < conv_bf16_blocks(h, w) || nblk > 256) return hipErrorInvalidValue;
    return dispatch_conv<2>(ConvArgs{(const uint16_t*)in, (const uint16_t*)wpk, bias, nullptr, (uint16_t*)d8, h, w,
                                     nblk, st, hd, ConvFirst{}},
                            nblk, s);
}

hipError_t launch_conv_fwd_first(const ConvFirst& cf, const void* wpk, const float* bias, void* out,
                                 uint16_t* mbits, int h, int w, const DevState* st, hipStream_t s) {
    const int nb = conv_bf16_blocks(h, w);
    return dispatch_conv<4>(ConvArgs{nullptr, (const uint16_t*)wpk, bias, mbits, (uint16_t*)out, h, w, nb, st,
                                     ConvHead{}, cf},
                            nb, s);
}

hipError_t launch_conv_fwd_val(const void* in, const void* wpk, const float* bias, const ConvHead& hd, int h, int w,
                               DevState* st, double* vtrace, hipStream_t s) {
    const int nb = conv_bf16_blocks(h, w);
    hipError_t e = dispatch_conv<3>(ConvArgs{(const uint16_t*)in, (const uint16_t*)wpk, bias, nullptr, nullptr, h, w,
                                             nb, (const DevState*)st, hd, ConvFirst{}},
                                    nb, s);
    if (e != hipSuccess) return e;
    return launch_decide(hd.lpart, nb, (long long)h * w, st, vtrace, s);
}

hipError_t launch_conv_bwd(const void* dlt, const void* wpk, const void* mask, void* out, int bf16, int h, int w,
                           const DevState* st, hipStream_t s) {
    dim3 grid((w + kTile - 1) / kTile, (h + kTile - 1) / kTile);
    if (bf16) {
        const int nb = conv_bf16_blocks(h, w);
        return dispatch_conv<1>(ConvArgs{(const uint16_t*)dlt, (const uint16_t*)wpk, nullptr,
                                         (uint16_t*)const_cast<void*>(mask), (uint16_t*)out, h, w, nb, st, ConvHead{},
                                         ConvFirst{}},
                                nb, s);
    }
    if (launch_recorder()) return hipErrorNotSupported;
    hipLaunchKernelGGL(k_conv_f32<1>, grid, dim3(256), 0, s, (const float*)dlt, (const float*)wpk,
                       (const float*)nullptr, (const float*)mask, (float*)out, h, w, st);
    return hipGetLastError();
}

int head_fused_blocks(int h, int w) { return conv_bf16_blocks(h, w); }

int wgrad_splits(int h, int w, int bf16, int cap) {
    const int tiles = ((w + kTile - 1) / kTile) * ((h + kTile - 1) / kTile);
    if (cap <= 0) cap = bf16 ? kMaxSplitBf16 : kMaxSplit;
    return tiles < cap ? tiles : cap;
}

hipError_t launch_wgrad(const void* src, const void* dlt, float* part, int nsplit, int bf16, int h, int w,
                        const DevState* st, hipStream_t s) {
    if (bf16) {
        const WgradArgs a{(const uint16_t*)src, (const uint16_t*)dlt, part, h, w, st};
        if (launch_recorder()) return record_launch(KK_WGRAD, &a, sizeof(a), 4 * nsplit, (long long)h * w, 1);
        hipLaunchKernelGGL(k_wgrad_bf16, dim3(4 * nsplit), dim3(512), 0, s, a);
        return hipGetLastError();
    }
    if (launch_recorder()) return hipErrorNotSupported;
    hipLaunchKernelGGL(k_wgrad_f32, dim3(nsplit), dim3(256), 0, s, (const float*)src, (const float*)dlt, part, h, w,
                       st);
    return hipGetLastError();
}

hipError_t launch_group_conv(int kind, GroupView v, int grid, hipStream_t s) {
    switch (kind) {
        case KK_CONV_FWD: hipLaunchKernelGGL(k_conv_bf16_group<0>, dim3(grid), dim3(512), 0, s, v); break;
        case KK_CONV_DGRAD: hipLaunchKernelGGL(k_conv_bf16_group<1>, dim3(grid), dim3(512), 0, s, v); break;
        case KK_CONV_HEAD: hipLaunchKernelGGL(k_conv_bf16_group<2>, dim3(grid), dim3(512), 0, s, v); break;
        case KK_CONV_VAL: hipLaunchKernelGGL(k_conv_bf16_group<3>, dim3(grid), dim3(512), 0, s, v); break;
        case KK_CONV_FIRST: hipLaunchKernelGGL(k_conv_bf16_group<4>, dim3(grid), dim3(512), 0, s, v); break;
        case KK_WGRAD: hipLaunchKernelGGL(k_wgrad_bf16_group, dim3(grid), dim3(512), 0, s, v); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace n2f
