// Internal interfaces shared by the host runtime (n2f_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

#include "n2f.h"

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
    int cout[kLayers + 1];    // output channels of layer l (1 for the head)
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
int wgrad_splits(int h, int w, int bf16, int cap = 0);   // cap 0: kMaxSplitBf16 / kMaxSplit
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

// ---------------------------------------------------------------------------
// Grouped launches: one launch of a kernel covers the same launch of many
// runs (the images of a batch at the same step of their epochs).  Each run's
// launch is a range of "virtual blocks", exactly the blocks its own launch
// would have; a grouped kernel's blocks walk the virtual blocks of all runs
// (block b takes b, b + grid, ...) and run each one as the run's own kernel
// would, so a run's results are the same bits grouped or alone.
//
// While a Recorder is installed on the calling thread, the launchers below
// record (kind, grid, arguments) instead of launching: the host runtime
// records one epoch per run and lays the records out as per-run argument
// tables in device memory.
// ---------------------------------------------------------------------------
enum KernelKind : int {
    KK_CONV_FWD = 0,   // k_conv_bf16<0>: 64->64 forward
    KK_CONV_DGRAD,     // k_conv_bf16<1>: data gradient
    KK_CONV_HEAD,      // k_conv_bf16<2>: last forward layer + training head
    KK_CONV_VAL,       // k_conv_bf16<3>: last validation layer + head
    KK_CONV_FIRST,     // k_conv_bf16<4>: first layer (one channel) fused into layer 2
    KK_WGRAD,          // k_wgrad_bf16
    KK_CONV1_C1,       // k_conv1<C, BF16>, C = 1, 2, 3
    KK_CONV1_C2,
    KK_CONV1_C3,
    KK_WGRAD1_C1,      // k_wgrad1<C, BF16>, C = 1, 2, 3
    KK_WGRAD1_C2,
    KK_WGRAD1_C3,
    KK_ADAM,           // k_adam
    KK_DECIDE,         // k_decide
    KK_ACCUM,          // k_accumulate
    KK_COUNT
};
static_assert(KK_COUNT == N2F_GROUP_KINDS, "grouped kinds of the header");
constexpr int kArgStride = 512;   // bytes per run of a grouped launch's argument table

struct LaunchRec {
    int kind;
    int grid;                     // virtual blocks of this run's launch
    long long npix;               // pixels the launch processes (kernel timing)
    int cost;                     // relative work of one virtual block (balancing)
    alignas(16) unsigned char args[kArgStride];
};
struct Recorder {
    std::vector<LaunchRec> recs;
};
// The calling thread's recorder (nullptr: launch directly).
Recorder*& launch_recorder();
hipError_t record_launch(int kind, const void* args, size_t bytes, int grid, long long npix, int cost);

// A grouped launch: prefix = {n, 0, g_0, g_0 + g_1, ..., total} (the runs'
// virtual block counts), args = n argument blocks of kArgStride bytes,
// starts = the first virtual block of each block of a launch whose blocks
// take consecutive ranges (grid + 1 entries, balanced by cost).
constexpr int kMaxGroupGrid = N2F_MAX_GROUP_GRID;
struct GroupView {
    const unsigned char* args;
    const int* prefix;
    const int* starts;
};
// One run's argument block of a grouped launch, read by every lane of the
// block (one cache line) and moved word by word to scalar registers: loaded
// as ordinary vector loads they would hold the run's pointers in vector
// registers for the whole kernel.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "argument blocks are whole 4-byte words");
    constexpr int kWords = sizeof(T) / 4;
    union {
        T t;
        int w[kWords];
    } u;
    const int* src = reinterpret_cast<const int*>(p);
#pragma unroll
    for (int i = 0; i < kWords; ++i) u.w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return u.t;
}
// A pointer read out of an argument block carries no address space, so
// loads and stores through it compile to flat instructions.  Those count as
// LDS operations as well, and every wait for an LDS read then also waits
// for the global loads in flight.  Every pointer of an argument block
// points into device memory; the hot loads and stores go through
// `as_global` pointers, which compile to global instructions.  (The host
// pass of a HIP source parses device functions too; there the qualifier is
// empty.)
#if defined(__HIP_DEVICE_COMPILE__)
#define N2F_GLOBAL __attribute__((address_space(1)))
#else
#define N2F_GLOBAL
#endif
template <class T>
__device__ __forceinline__ const N2F_GLOBAL T* as_global(const T* p) {
    return (const N2F_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ N2F_GLOBAL T* as_global(T* p) {
    return (N2F_GLOBAL T*)p;
}
// Buffer resource over device memory from `base` (which may lie before the
// data: only base + offset is accessed).  Reads at offset kBufOut return
// zeros and writes there are dropped, so a tile's loads and stores outside
// the image need no branch: every lane issues the same accesses, which the
// compiler can count (it then waits for exactly the ones a value needs).
constexpr uint32_t kBufOut = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
// Barrier for LDS traffic: waits for this wave's LDS operations, then for
// the other waves of the block.  __syncthreads() also waits for the wave's
// global loads in flight (its release fence covers global memory, and the
// loads share a counter with the stores), so a tile loaded ahead across it
// would always be waited for at the barrier.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// Wait until at most N of this wave's vector-memory operations are in
// flight (they complete in order for loads).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    // s_waitcnt fields: vmcnt[3:0], expcnt[6:4] (7: no wait), lgkmcnt[11:8] (15: no wait), vmcnt[5:4] at [15:14]
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
// Device side: walk the virtual blocks of a grouped launch, block b taking
// b, b + gridDim.x, ...; f(run, virtual block, virtual blocks of that run).
// The barrier frees the block's shared memory for the next virtual block.
template <class F>
__device__ __forceinline__ void for_group_blocks(const GroupView& g, F&& f) {
    const int n = g.prefix[0];
    const int* pre = g.prefix + 1;
    const int total = pre[n];
    int s = 0;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
        while (vb >= pre[s + 1]) ++s;
        __syncthreads();
        f(s, vb - pre[s], pre[s + 1] - pre[s]);
    }
}
// Launch kind `kind` over a group with `grid` blocks (n2f_conv.hip holds the
// 3x3 kinds, n2f_kernels.hip the others).
hipError_t launch_group_conv(int kind, GroupView v, int grid, hipStream_t s);
hipError_t launch_group_misc(int kind, GroupView v, int grid, hipStream_t s);
inline hipError_t launch_group(int kind, GroupView v, int grid, hipStream_t s) {
    return (kind <= KK_WGRAD) ? launch_group_conv(kind, v, grid, s) : launch_group_misc(kind, v, grid, s);
}

// Record one epoch (the four training steps in the configured pair order,
// then the validation) of network `net` of run r: the launches it would
// make, in order.  BF16 runs only (N2F_EINVAL otherwise).
n2f_status record_epoch(n2f_run* r, int net, std::vector<LaunchRec>* out);
hipStream_t run_stream(n2f_run* r);
// Kernel timing is on (n2f_profile_begin): grouped runs then poll every epoch,
// so that no timed launch covers a network that has already finished.
bool profiling_on();

// Blocks of a grouped launch of each kind (a tuning parameter: results do
// not depend on it).
int group_grid(int kind);
void set_group_grid(int kind, int grid);
// Kinds whose grouped blocks take consecutive, cost-balanced ranges of
// virtual blocks (GroupView::starts); the others take b, b + grid, ...
inline bool group_contiguous(int kind) { return kind <= KK_CONV_FIRST; }

// Many runs that advance together: every launch of an epoch is one grouped
// launch over all of them, and a whole epoch is one recorded graph.  The
// runs share the group's stream (they must have been created on it) and
// must have the same channel count.  The argument tables live in caller
// device memory of table_bytes(cap) bytes and are rewritten (between
// epochs, on the stream) when a run joins, leaves or moves to its next
// network; the recorded graph stays valid.
class Group {
   public:
    static constexpr int kMaxPos = 128;   // launches per epoch
    static size_t table_bytes(int cap);
    Group(int cap, char* d_tab, hipStream_t s) : cap_(cap), d_tab_(d_tab), stream_(s) {}
    ~Group();
    Group(const Group&) = delete;
    Group& operator=(const Group&) = delete;
    // Add network `net` of run r under `tag` (the caller's handle).
    n2f_status add(n2f_run* r, int net, int tag);
    // The run under `tag` moves on to network `net`.
    n2f_status set_net(int tag, int net);
    // Drop `tag`; the caller synchronises the stream before it reuses the
    // run's workspace.
    void remove(int tag);
    int size() const { return (int)slots_.size(); }
    // Queue `epochs` epochs of every run (graph replays, or direct launches
    // in the epochs the kernel profiler times).
    n2f_status launch(int epochs);
    hipStream_t stream() const { return stream_; }
    // The next epoch this process launches runs as timed direct launches
    // (kernel timing is on and this is one epoch in `every`).
    static bool next_epoch_timed();

   private:
    struct Slot {
        int tag;
        n2f_run* run;
        int net;
        std::vector<LaunchRec> recs;
    };
    size_t pos_bytes() const;
    n2f_status upload();
    n2f_status enqueue_all(hipStream_t s, bool timed);
    int cap_;
    char* d_tab_;
    hipStream_t stream_;
    std::vector<Slot> slots_;
    std::vector<int> kinds_;
    std::vector<long long> npix_;          // pixels per launch over all runs
    std::vector<unsigned char> host_;      // staging copy of the tables
    bool dirty_ = true;
    hipStream_t cap_stream_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    int exec_grid_[KK_COUNT] = {};
};

// Networks of other widths than 64 (n2f_generic.hip): generic 3x3
// convolution (mode 0 forward + bias + ReLU, mode 1 data gradient masked by
// [act > 0]) from a packed operand, weight-gradient partials (nsplit copies of
// 9 CI CO + CO floats), the heads (train: d8, head partial rows of CI + 1 and
// loss partials; validation: y and squared-error partials), Adam from the
// partials, and the packed operands of one layer.  in_fp32 / w_fp32 mark the
// first layer of a BF16 run (FP32 image and weights).
hipError_t launch_gconv(const void* in, int CI, bool in_fp32, const void* wp, bool w_fp32, int CIpad,
                        const float* bias, const void* act, void* out, int CO, int mode, int bf16, int h, int w,
                        const DevState* st, hipStream_t s);
hipError_t launch_gwgrad(const void* src, int CI, bool src_fp32, const void* dlt, int CO, float* part, int nsplit,
                         int bf16, int h, int w, const DevState* st, hipStream_t s);
hipError_t launch_ghead(const void* a8, int CI, const float* tgt, int C, int k, const float* w9, void* d8, float* y,
                        float* part, double* lpart, int nblk, int train, int bf16, long long npix, DevState* st,
                        hipStream_t s);
hipError_t launch_gadam(float* theta, float* m, float* v, float* g, const float* part, const ParamTable& pt, float lr,
                        double beta1, double beta2, float eps, const double* lpart, int nloss, long long loss_npix,
                        DevState* st, hipStream_t s);
hipError_t launch_gpack(const float* theta, int off, int cin, int cout, int CIpad, void* fwd, void* bwd, bool w_fp32,
                        const DevState* st, hipStream_t s);

// Message returned by n2f_last_error() on the calling thread.
void set_last_error(const char* msg);
inline void set_last_error(const std::string& msg) { set_last_error(msg.c_str()); }

}  // namespace n2f
