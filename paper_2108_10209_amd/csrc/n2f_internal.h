// Internal interfaces shared by the host runtime (n2f_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

namespace n2f {

constexpr int kWidth = 64;        // channels of every hidden layer
constexpr int kLayers = 8;        // 3x3 conv layers
constexpr int kTaps = 9;
constexpr int kConvW = kTaps * kWidth * kWidth;   // weights of a 64->64 layer
constexpr int kConvN = kConvW + kWidth;           // ... plus its bias
constexpr int kHeadN = kWidth + 1;                // 1x1 head: 64 weights + bias
constexpr int kMaxSplit = 256;                    // max pixel splits of a weight gradient
constexpr int kMaxSplitBf16 = 64;                 // ... of the BF16 64->64 one (4 blocks per split)
constexpr int kMaxHeadSplit = 1024;               // max blocks of the training head

// Per-network state that lives in device memory.  The stopping rule is
// decided on the device so that whole epochs can be queued without a host
// round trip; every epoch kernel returns at once when `done` is set.
struct DevState {
    double best;          // best validation score so far (+inf at start)
    double last_v;        // score of the last validation
    double loss;          // mean BCE of the last training step
    long long t;          // Adam steps taken
    int epoch;            // validations done
    int best_epoch;       // epoch of `best` (1-based), 0 before the first
    int n_since;          // validations since the best one
    int improved;         // last validation improved on the best
    int done;             // network finished (rule fired, cap hit, or numeric failure)
    int capped;           // finished by max_epochs
    int acc;              // the last validation produced an output to fold into the running sum
    int nonfinite;        // a non-finite score was seen
    int patience, max_epochs, fixed_epochs;
};

// Where each trainable tensor of one network sits.  The internal ("tap
// major") layout of a 3x3 layer is W[t][ci][co] followed by b[co]; the head
// is w9[c] followed by b9.  Weight-gradient partial sums of layer l use the
// same per-layer layout, one copy per pixel split.
struct ParamTable {
    int off[kLayers + 1];     // offset of layer l (0-based, 8 = head) in theta
    int n[kLayers + 1];       // floats of layer l
    int cin[kLayers + 1];     // input channels of layer l
    int split[kLayers + 1];   // number of partial copies of layer l
    long long poff[kLayers + 1];  // offset of layer l's partials in the partial buffer
    int total;                // parameters of one network
};

// Packed convolution operands for layers 2..8 (index l-1 = 1..7).  For the
// FP32 kernels, per layer 9*64*64 floats:
//   fwd[t][ci/4][co][ci%4]   = W[t][ci][co]
//   bwd[t][co/4][ci][co%4]   = W[8-t][ci][co]     (flipped taps, transposed)
// For BF16, per layer 9*64*64 bf16:
//   fwd[t][ci/8][co][ci%8], bwd[t][co/8][ci][co%8].
constexpr int kPackN = kTaps * kWidth * kWidth;

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All return hipError_t of the
// launch.  `st` may be null for kernels run outside an epoch.
// ---------------------------------------------------------------------------
hipError_t launch_minmax(const float* x, long long n, float* part, int nblk, unsigned* counter,
                         float* lohi, int* nonfinite, hipStream_t s);
hipError_t launch_prepare(const float* x, int H, int W, int C, const float* lohi,
                          float* xs, float* ue, float* uo, float* le, float* lo, int quad, hipStream_t s);
// x[0..3]: the noisy downsamples; t[0..3]: the clean ones on entry, the
// pair targets on exit; n values per image.
hipError_t launch_exact_targets(const float* const* x, float* const* t, long long n, hipStream_t s);
// out[p] = max over z < nz of stack[z * npix + p]; nz >= 1, npix >= 1.
hipError_t launch_max_project(const float* stack, int nz, long long npix, float* out, hipStream_t s);
hipError_t launch_init_state(DevState* st, int patience, int max_epochs, int fixed_epochs, hipStream_t s);
hipError_t launch_pack(const float* theta, const ParamTable& pt, float* fwd, float* bwd,
                       uint16_t* fwd16, uint16_t* bwd16, hipStream_t s);
// BF16 runs keep a ReLU bit mask per stashed activation (8 bytes per pixel,
// see k_conv_bf16); the forward launchers write it when `mbits` is given and
// the BF16 data gradient takes it as `mask`.  FP32 runs pass mbits = NULL
// and give the data gradient the FP32 activation itself as `mask`.
hipError_t launch_conv1(const float* in, int C, const float* w1, const float* b1, void* out, uint16_t* mbits,
                        int bf16, int h, int w, const DevState* st, hipStream_t s);
hipError_t launch_conv_fwd(const void* in, const void* wpk, const float* bias, void* out, uint16_t* mbits,
                           int bf16, int h, int w, const DevState* st, hipStream_t s);
hipError_t launch_conv_bwd(const void* dlt, const void* wpk, const void* mask, void* out, int bf16,
                           int h, int w, const DevState* st, hipStream_t s);
// BF16 path: the last 3x3 forward layer with the training head in its
// epilogue (z = w9 . a8 + b9, the mean-BCE gradient, d8 = dL/dz w9 [a8 > 0],
// one partial row of dW9, db9 and of the loss per block); a8 itself is not
// stored.  The grid is nblk blocks (>= head_fused_blocks(h, w)), one head
// partial row each, so every pair shape fills the same nblk rows.
struct ConvHead {
    const float* w9;     // head weights, then b9
    const float* tgt;    // target image (validation: the noisy image), C channels per pixel
    float* part;         // nblk x kHeadN partial sums of dW9, db9 (training)
    double* lpart;       // nblk partial sums of the BCE (training) or of the squared error (validation)
    float* y;            // validation: the network's output image
    DevState* st;        // training: its step counter counts the Adam step that follows
    int C, k;            // target channels, and the one this network predicts
    float invP;          // training: 1 / pixels of the pair
};
// BF16 path, one input channel: the first layer (3x3, 1 -> 64, bias, ReLU)
// computed inside the layer-2 forward kernel from a 20 x 20 input halo per
// tile, straight into its staged LDS halo; a1 and its ReLU bit mask are
// still stored (the backward pass reads them) unless the pointers are NULL.
struct ConvFirst {
    const float* x;      // input image, h x w, one channel
    const float* w1;     // first-layer weights [t][co] (9 x 64)
    const float* b1;     // first-layer biases (64)
    uint16_t* a1;        // a1 out (BF16, h x w x 64), or NULL
    uint16_t* m1;        // a1's ReLU bit mask out (8 bytes per pixel), or NULL
};
hipError_t launch_conv_fwd_first(const ConvFirst& cf, const void* wpk, const float* bias, void* out,
                                 uint16_t* mbits, int h, int w, const DevState* st, hipStream_t s);
int head_fused_blocks(int h, int w);   // blocks of the BF16 convolution grid at h x w
hipError_t launch_conv_fwd_head(const void* in, const void* wpk, const float* bias, void* d8, const ConvHead& hd,
                                int nblk, int h, int w, const DevState* st, hipStream_t s);
// The same for the validation pass: y = sigmoid(z) and one partial sum of
// (y - x)^2 per block, in FP64 (then the stopping decision, as after
// launch_head_val); a8 is not stored.
hipError_t launch_conv_fwd_val(const void* in, const void* wpk, const float* bias, const ConvHead& hd, int h, int w,
                               DevState* st, double* vtrace, hipStream_t s);
// Fixed-order sum of nblk validation partials and the stopping decision.
hipError_t launch_decide(const double* vpart, int nblk, long long npix, DevState* st, double* vtrace, hipStream_t s);
int wgrad_splits(int h, int w, int bf16);
hipError_t launch_wgrad(const void* src, const void* dlt, float* part, int nsplit, int bf16,
                        int h, int w, const DevState* st, hipStream_t s);
hipError_t launch_wgrad1(const float* in, int C, const void* dlt, float* part, int nsplit, int bf16,
                         int h, int w, const DevState* st, hipStream_t s);
int head_splits(long long npix);
hipError_t launch_head_train(const void* a8, const float* tgt, int C, int k, const float* w9,
                             const float* b9, void* d8, float* part, double* lpart, int nsplit,
                             int bf16, long long npix, DevState* st, hipStream_t s);
hipError_t launch_head_val(const void* a8, const float* xs, int C, int k, const float* w9,
                           const float* b9, float* y, double* vpart, int nblk, int bf16,
                           long long npix, DevState* st, double* vtrace, hipStream_t s);
hipError_t launch_accumulate(const float* y, float* S, float* ybest, long long npix, DevState* st,
                             hipStream_t s);
hipError_t launch_finalize(const float* y, const float* S, const float* ybest, const float* lohi,
                           float* out, long long npix, const DevState* st, hipStream_t s);
hipError_t launch_adam(float* theta, float* m, float* v, float* g, const float* part,
                       const float* ginj, const ParamTable& pt, float lr, double beta1,
                       double beta2, float eps, float* fwd, float* bwd, uint16_t* fwd16,
                       uint16_t* bwd16, const double* lpart, int nloss, long long loss_npix,
                       DevState* st, hipStream_t s);
hipError_t launch_extract(const float* src, int h, int w, int C, float* out_chw, hipStream_t s);

// Message returned by n2f_last_error() on the calling thread.
void set_last_error(const char* msg);
inline void set_last_error(const std::string& msg) { set_last_error(msg.c_str()); }

}  // namespace n2f
