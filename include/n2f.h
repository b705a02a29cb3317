/*
 * n2f.h -- C ABI of the Noise2Fast per-image train-and-denoise library for
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the one stated in the Theoretical Background of Noise2Fast
 * (Lequyer et al., arXiv 2108.10209): given one noisy image x = s + n, find a
 * network f with f(x) ~ s, using nothing but x.  The method (Methods section,
 * "Noise2Fast Implementation Details"):
 *   1. standardise x (no clipping) and checkerboard-downsample it into four
 *      half-size images (the "up" and "left" downsample equations, Fig. 1);
 *   2. train a small feed-forward net (eight 3x3 conv+ReLU layers of width
 *      64, then a 1x1 conv and a sigmoid; Fig. 2a) on the four (input,
 *      target) pairs of the Methods table, one pair per Adam step (lr 1e-3,
 *      batch size 1), with a binary cross-entropy loss;
 *   3. after every epoch run the full image through the net and take the
 *      MSE against the noisy input; stop once 100 epochs pass without a new
 *      best score and return the mean of the last 100 validation outputs.
 * Multi-channel images train one single-output network per channel, each
 * seeing every input channel (Fig. 2a caption).
 *
 * Conventions
 *  - Every call returns an n2f_status: 0 success, < 0 error, > 0 warning.
 *    n2f_last_error() returns a message for the calling thread's last error.
 *    No exception or abort crosses the ABI.
 *  - Images are FP32, planar C x H x W (CHW), in DEVICE memory owned by the
 *    caller.  The library never frees or keeps them beyond a run's life.
 *  - All device memory a run uses comes from one caller-provided device
 *    workspace of at least n2f_workspace_bytes() bytes; the library makes
 *    no device allocation of its own.  The workspace must stay alive and
 *    untouched until n2f_run_destroy().
 *  - Work is queued on the caller's HIP stream.  Calls marked "synchronises"
 *    wait for that stream; the others return once the work is queued.
 *  - A run is not thread-safe; distinct runs are independent.
 *  - Parameter vectors exchanged with the host use the canonical layout of
 *    one output-channel network: W1 (w1, C, 3, 3), b1 (w1), W2..W8
 *    (w_l, w_{l-1}, 3, 3) each followed by its bias (w_l), W9 (1, w8, 1, 1),
 *    b9 (1), each flattened in C order (n2f_param_count() floats in total);
 *    w_l = 64 for the default network.
 */
#ifndef N2F_H
#define N2F_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int n2f_status;

#define N2F_OK          0
#define N2F_EINVAL     (-1)   /* bad argument: size, pointer, non-finite input, config */
#define N2F_ENOMEM     (-2)   /* workspace smaller than n2f_workspace_bytes() */
#define N2F_EDEVICE    (-3)   /* a HIP runtime call failed */
#define N2F_ESTATE     (-4)   /* call not valid in the run's current state */
#define N2F_ENUMERIC   (-5)   /* a validation score became NaN or infinite */
#define N2F_ECANCELED  (-6)   /* a served request was cancelled before it finished */
#define N2F_WCONSTANT   1     /* constant image: returned unchanged, nothing trained */
#define N2F_WCAPPED     2     /* max_epochs reached before the stopping rule fired */

#define N2F_FP32 0            /* convolutions on FP32 MFMA */
#define N2F_BF16 1            /* convolutions on BF16 MFMA, FP32 accumulate, FP32 master weights */

#define N2F_DS_CHECKERBOARD 0 /* the paper's checkerboard downsamples (Fig. 1) */
#define N2F_DS_QUAD         1 /* ablation (Methods, Ablation Study; Table 1 "Quad"): 2x2 blocks */

typedef struct n2f_config {
    int    n_layers;          /* 3x3 conv layers; only 8 is supported */
    int    width;             /* channels of every 3x3 layer when widths[] is all zero (16..256, multiple of 16) */
    float  lr;                /* Adam step size (Methods: 1e-3) */
    float  eps;               /* Adam epsilon (Kingma and Ba default 1e-8) */
    double beta1, beta2;      /* Adam moment decays (0.9, 0.999); double so that 1 - beta is exact to FP32 */
    int    patience;          /* epochs without a new best before stopping (Methods: 100) */
    int    max_epochs;        /* safety cap (not in the paper); >= 1 */
    int    fixed_epochs;      /* > 0: run exactly this many epochs, output the last validation output */
    int    pair_order[4];     /* order of the four training pairs within an epoch */
    int    precision;         /* N2F_FP32 or N2F_BF16 */
    unsigned long long init_seed; /* SplitMix64 seed of the initial weights */
    int    use_graph;         /* n2f_run_epochs replays one recorded HIP graph per epoch */
    int    downsample;        /* N2F_DS_CHECKERBOARD or N2F_DS_QUAD (training pairs only) */
    int    exact_targets;     /* 1: "Exact" ablation; the run waits for n2f_run_set_clean() */
    int    widths[8];         /* per-layer output channels (16..256, multiples of 16), e.g. the Methods'
                                 own 32, 32, 64, 64, 128, 128, 256, 256; all zero: every layer `width`.
                                 Width 64 throughout runs on the tuned kernels; any other widths on generic
                                 FP32-MFMA kernels (BF16 storage in BF16 runs), not in grouped launches */
    int    wgrad_splits;      /* most pixel splits of a 64->64 weight gradient (1..256); 0: 64 (BF16) or
                                 256 (FP32).  Fewer splits write and re-read fewer partial rows (each is
                                 9*64*64+64 floats) at the cost of fewer blocks per launch; the split count
                                 fixes the order of the gradient's sums, so runs compare bit for bit only
                                 at the same value */
} n2f_config;

typedef struct n2f_run n2f_run;

/* Fill *cfg with the paper's settings: 8 layers of width 64 (widths[] zero), Adam lr 1e-3,
 * betas 0.9/0.999, eps 1e-8, patience 100, max_epochs 2000, early stopping,
 * pairs in table order, FP32, seed 0, epochs replayed as HIP graphs,
 * checkerboard downsampling, plain targets. */
void n2f_config_default(n2f_config* cfg);

/* Message describing the calling thread's most recent error ("" if none). */
const char* n2f_last_error(void);

/* Number of parameters of one output-channel network for C input channels. */
n2f_status n2f_param_count(int C, const n2f_config* cfg, size_t* count);

/* Host-only: the initial weights the library draws for a run, written to
 * host buffer theta (C * n2f_param_count floats, network k at offset
 * k * count).  Every weight and bias of a layer is U(-1/sqrt(fan_in),
 * +1/sqrt(fan_in)) (fan_in = Cin*kh*kw; the paper leaves initialisation
 * open); value i of network k is (2u - 1) * bound rounded once to FP32,
 * with u the top 53 bits of SplitMix64 output number k*count + i of `seed`. */
n2f_status n2f_init_params(int C, const n2f_config* cfg, unsigned long long seed, float* theta);

/* Device workspace bytes a run on an H x W x C image needs (H, W >= 2,
 * 1 <= C <= 3).  This figure is also the unit of HBM admission when runs
 * share a GPU.  cfg->exact_targets adds room for four target images. */
n2f_status n2f_workspace_bytes(int H, int W, int C, const n2f_config* cfg, size_t* bytes);

/* Create a run: validates arguments, standardises the image (per-image
 * min-max to [0, 1], no clipping), builds the four downsamples (checkerboard
 * or, with cfg->downsample = N2F_DS_QUAD, the 2x2-block images; even sizes,
 * an odd last row/column is left out of them only) and draws
 * the initial weights from cfg->init_seed.  d_in: device CHW image, read
 * during this call only.  Synchronises.  Returns N2F_WCONSTANT for a
 * constant image (the run then only supports n2f_result, which copies the
 * input), N2F_EINVAL for non-finite input. */
n2f_status n2f_run_create(n2f_run** run, const float* d_in, int H, int W, int C,
                          const n2f_config* cfg, void* d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* Release the run's host state.  The workspace may be reused afterwards. */
n2f_status n2f_run_destroy(n2f_run* run);

/* One training step of network `net` (0 <= net < C) on pair `pair`
 * (0: up-even -> up-odd, 1: up-odd -> up-even, 2: left-even -> left-odd,
 * 3: left-odd -> left-even; the Methods table): forward pass, BCE against
 * channel `net` of the target, backward pass, one Adam step.  Queued.
 * With N2F_DS_QUAD the pairs are the 2x2 blocks' diagonals (the paper does
 * not state them): 0: TL -> BR, 1: BR -> TL, 2: TR -> BL, 3: BL -> TR.
 * N2F_ESTATE for an exact-target run before n2f_run_set_clean(). */
n2f_status n2f_train_step(n2f_run* run, int net, int pair);

/* Validation of network `net` after an epoch: full-image forward pass, MSE
 * against channel `net` of the standardised input summed in FP64, then the
 * stopping rule (strict improvement resets the running sum of outputs;
 * otherwise the output is added).  Synchronises and reports the score, whether
 * it improved on the best and whether the network is finished.  Any pointer
 * may be NULL.  Returns N2F_ENUMERIC if the score is not finite. */
n2f_status n2f_validate(n2f_run* run, int net, double* v, int* improved, int* done);

/* Run whole epochs (four steps in cfg->pair_order, then validation) of
 * network `net` until it is finished or `max_epochs_now` epochs have run;
 * the device decides the stopping rule and the host polls it every few
 * epochs.  *done (may be NULL) reports whether the network finished.
 * Synchronises.  Returns N2F_WCAPPED when the run hit cfg->max_epochs. */
n2f_status n2f_run_epochs(n2f_run* run, int net, int max_epochs_now, int* done);

/* Write the denoised image (CHW, input units: lo + (hi - lo) * output) to
 * device buffer d_out: per channel the mean of the outputs since the best
 * epoch, the best output if none followed it, or the last output in
 * fixed-epoch mode.  Queued. */
n2f_status n2f_result(n2f_run* run, float* d_out);

/* One-shot denoise: create, train every network to its stopping rule,
 * write d_out, destroy.  Synchronises.  N2F_EINVAL with
 * cfg->exact_targets (that ablation needs the clean image). */
n2f_status n2f_denoise(const float* d_in, float* d_out, int H, int W, int C,
                       const n2f_config* cfg, void* d_ws, size_t ws_bytes,
                       hipStream_t stream);

/* One-shot denoise for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and result as n2f_denoise, but the run's
 * workspace is a fixed array of N2F_NOALLOC_MAX_BYTES inside the library,
 * one per device it runs on, held until the process ends; the epochs run as
 * direct launches (no graph is instantiated).  No device memory, stream,
 * event or graph is created.  Runs on the current device (`stream` must
 * belong to it).  N2F_ENOMEM when n2f_workspace_bytes(H, W, C, cfg) exceeds
 * N2F_NOALLOC_MAX_BYTES (BF16 grayscale fits up to about 256 x 256);
 * N2F_ESTATE while kernel timing (n2f_profile_begin) is on.  Calls on one
 * device share the array and must not overlap: concurrent calls race.
 * Synchronises. */
#define N2F_NOALLOC_MAX_BYTES ((size_t)128 << 20)
n2f_status n2f_denoise_noalloc(const float* d_in, float* d_out, int H, int W, int C,
                               const n2f_config* cfg, hipStream_t stream);

/* "Exact" ablation (Methods, Ablation Study; Table 1 "Exact"; the ODD
 * approximation of the Theoretical Background): with the clean image known,
 * the target of pair (a -> b) becomes x_b - (s_b - s_a), i.e. the input's
 * signal plus the target's noise.  d_clean: device CHW image of the run's
 * size, read during this call only, standardised with the noisy image's
 * minimum and maximum; it must be finite (N2F_EINVAL otherwise).  Needs
 * cfg->exact_targets at creation (N2F_ESTATE otherwise); may be called again
 * to replace the targets.  Validation and the output are unchanged.
 * Synchronises. */
n2f_status n2f_run_set_clean(n2f_run* run, const float* d_clean);

/* Maximum-intensity projection along z (Methods, Fluorescence Microscopy
 * Images: the live-cell volumes are denoised as individual z-slices and
 * then max projected).  d_stack: device FP32, n_slices (>= 1) images of npix
 * (>= 1) values each, slice z at d_stack + z * npix (e.g. the per-slice
 * results of a batch, one channel, copied into one buffer); d_out: device
 * FP32, npix values, not overlapping the stack:
 * d_out[p] = max_z d_stack[z * npix + p].  A NaN loses to any number (fmax),
 * so only a pixel that is NaN in every slice projects to NaN.  N2F_EINVAL
 * for NULL pointers, sizes below 1 or overlapping buffers.  Queued. */
n2f_status n2f_max_project(const float* d_stack, int n_slices, long long npix, float* d_out,
                           hipStream_t stream);

/* ---- state exchange (checkpoint/resume and teacher-forced testing) ---- */

/* Copy network `net`'s parameters, Adam moments and step count to host
 * buffers (canonical layout, n2f_param_count floats each; any may be NULL).
 * Synchronises. */
n2f_status n2f_get_state(n2f_run* run, int net, float* theta, float* m, float* v, long long* t);

/* Overwrite network `net`'s parameters, moments and step count from host
 * buffers (NULL m or v means zeros).  Synchronises. */
n2f_status n2f_set_state(n2f_run* run, int net, const float* theta, const float* m,
                         const float* v, long long t);

/* Whole-network checkpoints (resume, or moving a run between processes):
 * everything network `net` carries from epoch to epoch -- parameters, Adam
 * moments and step, the stopping-rule state and validation history, the
 * running output sum and the best and last outputs -- as an opaque host blob
 * of n2f_checkpoint_bytes() bytes.  A run created from the same image with
 * the same configuration and loaded from it continues exactly as the saved
 * run would have (bit-identical results).  Loading checks the image size,
 * channel count, precision, downsampling, target mode and epoch cap of the
 * blob against the run (N2F_EINVAL on a mismatch or a short buffer); the
 * other settings (learning rate, pair order) are the loading run's.  An
 * exact-target run needs n2f_run_set_clean again.  Save and load
 * synchronise. */
n2f_status n2f_checkpoint_bytes(n2f_run* run, size_t* bytes);
n2f_status n2f_save_checkpoint(n2f_run* run, int net, void* host_buf, size_t bytes);
n2f_status n2f_load_checkpoint(n2f_run* run, int net, const void* host_buf, size_t bytes);

/* Gradient (canonical layout, host buffer) that the last Adam step of
 * network `net` used, and that step's mean BCE loss.  Synchronises. */
n2f_status n2f_get_grad(n2f_run* run, int net, float* g, double* loss);

/* Apply one Adam step to network `net` with the host gradient g (canonical
 * layout) instead of a computed one.  Synchronises. */
n2f_status n2f_debug_adam(n2f_run* run, int net, const float* g);

/* Stopping-rule state of network `net`: epochs validated, best epoch,
 * epochs since the best, best score; any pointer may be NULL.  Synchronises. */
n2f_status n2f_get_progress(n2f_run* run, int net, int* epoch, int* best_epoch,
                            int* since_best, double* best);

/* Validation scores of network `net`, epochs 1..n (n <= epochs run), to a
 * host buffer.  Synchronises. */
n2f_status n2f_get_history(n2f_run* run, int net, int n, double* v);

/* Per-image extremes used by the standardisation (exact min and max). */
n2f_status n2f_get_lohi(n2f_run* run, float* lo, float* hi);

/* Copy an intermediate image to device buffer d_out (CHW, FP32):
 * which = 0..3: the downsamples up-even (C x H' x W'/2), up-odd,
 * left-even (C x H'/2 x W'), left-odd (N2F_DS_QUAD: TL, BR, TR, BL, each
 * C x H'/2 x W'/2; pair p trains on image p); 4: the standardised image
 * (C x H x W); 5 + k: the last validation output of network k
 * (H x W, standardised units); 8 + p: the target image of pair p (the
 * partner downsample, or the "Exact" target, N2F_ESTATE before
 * n2f_run_set_clean; shape of image p).  Queued. */
n2f_status n2f_get_image(n2f_run* run, int which, float* d_out);

/* Queue `n_epochs` whole epochs of network `net` on the run's stream (the
 * recorded epoch graph when cfg->use_graph, captured on first use) without
 * waiting; epochs after the network finishes do nothing.  Queued. */
n2f_status n2f_run_launch_epochs(n2f_run* run, int net, int n_epochs);

/* Wait for the run's stream and report whether network `net` is finished
 * and how many epochs it has validated (either pointer may be NULL).
 * Returns N2F_ENUMERIC after a non-finite score, N2F_WCAPPED when the
 * network stopped at cfg->max_epochs.  Synchronises that stream only. */
n2f_status n2f_run_poll(n2f_run* run, int net, int* done, int* epochs);

/* ---- many independent images ----
 * A batch trains one run per image, each with its own weights, Adam state,
 * stopping rule and workspace slice.  Each run replays its own recorded
 * epoch graph on one of the batch's streams (images spread largest first
 * onto the least loaded), so the epochs of different images overlap on the
 * device; networks of a multi-channel image run one after the other.  The
 * host serves the streams in turn (waits for one, reads its images'
 * stopping rules, queues their next epochs) while the others run.  Images
 * may differ in size and channel count.  Every batch call is made between
 * epochs, so images join (n2f_batch_add) and leave (n2f_batch_remove) at
 * epoch boundaries while the others keep their state. */
typedef struct n2f_batch n2f_batch;

/* Workspace for a batch: the 256-byte aligned sum of the images' needs,
 * plus the launch tables of grouped mode (12 groups: 3 channel counts x up
 * to 4 streams). */
n2f_status n2f_batch_workspace_bytes(int n, const int* H, const int* W, const int* C, const n2f_config* cfg,
                                     size_t* bytes);

/* Create the runs; image i reads its device CHW input d_in[i] during this
 * call, after the work already queued on the caller's `stream` (the batch's
 * streams wait for it, so inputs produced there are complete).  d_ws: 256-byte
 * aligned device workspace of n2f_batch_workspace_bytes(), image i's slice
 * at the aligned prefix sum of the sizes before it, then the launch tables
 * of grouped mode; kept until destroy.
 * n_streams >= 1: the batch creates that many streams (default priority),
 * at most one per image, and each image replays its own epoch graph;
 * n_streams = 0: everything runs on `stream` itself, one image after
 * another; n_streams = N2F_BATCH_GROUPED (BF16 only): every launch of an
 * epoch is one grouped launch over all images of the same channel count,
 * whose blocks run each image's blocks exactly as its own launch would (the
 * same bits as the image alone), and one recorded graph per epoch replays
 * on `stream`; n_streams = -K, K = 2..4 (BF16 only): grouped launches on K
 * streams the batch creates, the images split between them by work
 * (pixels x channels, largest first), one group per channel count and
 * stream, so launches of different kinds overlap across the streams (the
 * same bits again); the streams are refed in turn, each as soon as its own
 * images' stopping rules are read.  While kernel timing is on
 * (n2f_profile_begin), each timed epoch of such a batch runs alone: its
 * stream waits for the others and they wait for it.  At most n + 64 images train at once (n2f_batch_add
 * beyond that returns N2F_ENOMEM).  Synchronises.  Constant images are finished at
 * once.  cfg->exact_targets is refused (N2F_EINVAL), here and by the
 * server. */
#define N2F_BATCH_GROUPED (-1)
n2f_status n2f_batch_create(n2f_batch** batch, int n, const float* const* d_in, const int* H, const int* W,
                            const int* C, const n2f_config* cfg, void* d_ws, size_t ws_bytes, int n_streams,
                            hipStream_t stream);

/* Join a new image between n2f_batch_run calls (an epoch boundary): its run
 * is created on the least loaded batch stream, reading the device CHW image
 * d_in after the work queued on the batch's caller stream, with its own
 * 256-byte aligned workspace d_ws of at least n2f_workspace_bytes(H, W, C)
 * bytes (owned by the caller, kept until the image is removed or the batch
 * destroyed).  *index (may be NULL) receives the image's index (n so far).
 * Synchronises.  N2F_ENOMEM for a workspace that is too small. */
n2f_status n2f_batch_add(n2f_batch* batch, const float* d_in, int H, int W, int C, void* d_ws, size_t ws_bytes,
                         int* index);

/* Image i leaves the batch between n2f_batch_run calls: its queued work
 * ends, its run is destroyed and its workspace slice is the caller's again;
 * the other images keep training unchanged.  Later calls on image i return
 * N2F_ESTATE (result, run_of, remove); n2f_batch_progress reports it
 * finished.  Synchronises image i's stream. */
n2f_status n2f_batch_remove(n2f_batch* batch, int i);

/* Run epochs of every unfinished image until all are finished or each has
 * run `max_epochs_now` more epochs; *n_active (may be NULL) reports the
 * images still training.  An image whose validation score turns non-finite
 * is finished as failed (its n2f_batch_result returns N2F_ENUMERIC) and the
 * others go on.  Synchronises every batch stream. */
n2f_status n2f_batch_run(n2f_batch* batch, int max_epochs_now, int* n_active);

/* Write image i's result (CHW, input units) to d_out.  Synchronises.
 * N2F_ENUMERIC, writing nothing, for an image that failed. */
n2f_status n2f_batch_result(n2f_batch* batch, int i, float* d_out);

/* The run of image i, owned by the batch (never destroy it), for state
 * exchange between n2f_batch_run calls: n2f_get_state / n2f_set_state,
 * n2f_get_progress, n2f_get_history (checkpoint and resume of one image). */
n2f_status n2f_batch_run_of(n2f_batch* batch, int i, n2f_run** run);

/* Epochs run (all networks together) and finished flag of image i. */
n2f_status n2f_batch_progress(n2f_batch* batch, int i, int* epochs, int* finished);

n2f_status n2f_batch_destroy(n2f_batch* batch);

/* ---- continuous-batching server ----
 * Requests queue in arrival order.  A request is admitted when fewer than
 * `max_active` runs are active and its workspace (n2f_workspace_bytes) fits
 * in a free range of the caller's device arena (first fit; strict arrival
 * order, so a large request is never overtaken).  Each n2f_server_step
 * admits what fits, queues `epochs` epochs of every active run on its
 * stream, and retires finished runs: their result is written to the
 * request's d_out, their arena range is freed, and their id is reported by
 * n2f_server_poll.  Runs therefore join and leave at epoch boundaries while
 * the others keep training.
 * With flags & N2F_SERVER_SIMULATE no device work is done: a request
 * finishes after `sim_epochs` epochs, which tests the admission and
 * bookkeeping logic on a machine without a GPU.
 * With flags & N2F_SERVER_GROUPED (BF16 only) every launch of an epoch is one
 * grouped launch over all active requests of the same channel count (as in
 * a grouped batch), replayed as one graph per epoch on the server's single
 * stream (n_streams is then ignored); the launch tables for max_active runs
 * per channel count take the first n2f_server_table_bytes(max_active)
 * bytes of the arena, and requests are admitted into the rest. */
#define N2F_SERVER_SIMULATE 1
#define N2F_SERVER_GROUPED  2
typedef struct n2f_server n2f_server;

n2f_status n2f_server_create(n2f_server** srv, const n2f_config* cfg, void* d_arena, size_t arena_bytes,
                             int n_streams, int max_active, int flags);

/* Arena bytes a grouped server keeps for its launch tables. */
n2f_status n2f_server_table_bytes(int max_active, size_t* bytes);

/* Queue a request.  d_in and d_out: device CHW images owned by the caller,
 * kept alive and untouched until the id is reported by n2f_server_poll.
 * `stream`: the caller's stream on which d_in is produced; admission reads
 * d_in only after the work queued there before this call (an event recorded
 * now).  When the id is reported, d_out is complete on the device.  The id
 * must not be queued or active already (N2F_EINVAL).  N2F_ENOMEM if the
 * request could never fit in the arena. */
n2f_status n2f_server_submit(n2f_server* srv, long long id, const float* d_in, float* d_out, int H, int W, int C,
                             int sim_epochs, hipStream_t stream);

/* Cancel a queued or active request: it leaves at once (an active run's
 * queued epochs end first, then its arena range is freed), d_out is not
 * written, and n2f_server_poll reports the id with N2F_ECANCELED.
 * N2F_EINVAL for an id that is neither queued nor active (e.g. finished).
 * Synchronises the request's stream if it is active. */
n2f_status n2f_server_cancel(n2f_server* srv, long long id);

/* One scheduling round as described above.  Synchronises the active
 * streams.  Reports active and queued request counts (pointers may be NULL). */
n2f_status n2f_server_step(n2f_server* srv, int epochs, int* n_active, int* n_queued);

/* Pop up to `max` finished ids (completion order) into ids; *n = count.
 * status (may be NULL) receives each request's final n2f_status. */
n2f_status n2f_server_poll(n2f_server* srv, long long* ids, int* status, int max, int* n);

/* Arena bytes in use and the largest free range. */
n2f_status n2f_server_memory(n2f_server* srv, size_t* used, size_t* largest_free);

n2f_status n2f_server_destroy(n2f_server* srv);

/* ---- kernel timing ----
 * While profiling is on, the launches of one epoch in `every` are issued
 * directly (not from the epoch's graph) and each run of consecutive launches
 * of an instrumented class is bracketed by two HIP events on the stream it
 * runs on.  Classes:
 *   N2F_K_CONV_FWD  64->64 forward convolution; a run is the 7 launches of
 *                   one forward pass (training or validation);
 *   N2F_K_BACKWARD  one 64->64 layer's backward, i.e. its weight-gradient
 *                   launch plus its data-gradient launch; a run is the 7
 *                   layers of one backward pass;
 *   N2F_K_ADAM      the fused gradient reduction + Adam launch.
 * n2f_profile_begin clears earlier records; n2f_profile_read synchronises
 * the recorded events and returns, for one class, the summed time of its
 * runs, the number of launches (pairs for N2F_K_BACKWARD) in them and the
 * pixels those launches processed.  Process-wide; not thread-safe. */
#define N2F_K_CONV_FWD 0
#define N2F_K_BACKWARD 1
#define N2F_K_ADAM     2
/* Grouped launches (a batch created with N2F_BATCH_GROUPED, or a server with
 * N2F_SERVER_GROUPED): each launch covers every image of the group and is
 * bracketed on its own; class N2F_K_GROUP + kind, pixels summed over the
 * images.  Kinds: 0 64->64 forward, 1 data gradient, 2 last layer with the
 * training head, 3 last layer with the validation head, 4 first layer fused
 * into layer 2, 5 64->64 weight gradient, 6-8 first layer (C = 1, 2, 3),
 * 9-11 first-layer weight gradient (C = 1, 2, 3), 12 Adam, 13 stopping rule,
 * 14 running output sum. */
#define N2F_K_GROUP   16
n2f_status n2f_profile_begin(int every);
n2f_status n2f_profile_read(int kernel_class, double* total_ms, long long* launches, long long* pixels);
n2f_status n2f_profile_end(void);

/* Launch geometry of grouped launches (tuning; no paper passage: how many
 * hardware blocks one grouped launch of a kind uses to walk the virtual
 * blocks of its images).  `kind` is a grouped kind 0..14 as listed above;
 * `grid` is 1..N2F_MAX_GROUP_GRID.  The geometry never changes results: each
 * virtual block computes the same values whichever hardware block runs it.
 * A change takes effect at the next epoch of every group (their captured
 * launches are recorded again).  Process-wide; not thread-safe with running
 * groups.  N2F_EINVAL for a kind or grid out of range. */
#define N2F_GROUP_KINDS 15
#define N2F_MAX_GROUP_GRID 1024
n2f_status n2f_group_grid_get(int kind, int* grid);
n2f_status n2f_group_grid_set(int kind, int grid);

#ifdef __cplusplus
}
#endif
#endif /* N2F_H */
