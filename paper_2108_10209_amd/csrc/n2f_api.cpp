// Host runtime of the Noise2Fast library: argument checks, workspace
// carving, weight initialisation, the per-step and per-epoch launch
// sequences, and state exchange.  See include/n2f.h for the contract.
#include "n2f.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "n2f_internal.h"

using namespace n2f;

namespace {

thread_local std::string g_err;

n2f_status fail(n2f_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define N2F_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(N2F_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// SplitMix64 (Steele, Lea and Flood 2014), counter form.
inline unsigned long long splitmix64(unsigned long long seed, unsigned long long n) {
    unsigned long long z = seed + (n + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Shapes of one network in canonical order: (cin, kernel taps) per layer.
struct CanonLayer {
    int cout, cin, taps;
};

// Per-layer output channels of the eight 3x3 layers: widths[] if set, else
// `width` for every layer.
struct Widths {
    int w[kLayers];
};
Widths eff_widths(const n2f_config* cfg) {
    Widths ew{};
    for (int l = 0; l < kLayers; ++l) ew.w[l] = cfg->widths[0] ? cfg->widths[l] : cfg->width;
    return ew;
}
bool is_default_width(const Widths& ew) {
    for (int l = 0; l < kLayers; ++l)
        if (ew.w[l] != kWidth) return false;
    return true;
}

std::vector<CanonLayer> canon_layers(int C, const Widths& ew) {
    std::vector<CanonLayer> v;
    int cin = C;
    for (int l = 0; l < kLayers; ++l) {
        v.push_back({ew.w[l], cin, kTaps});
        cin = ew.w[l];
    }
    v.push_back({1, cin, 1});
    return v;
}

ParamTable make_table(int C, const Widths& ew, int n1split, int nsplit, int hsplit) {
    ParamTable pt{};
    int off = 0;
    long long poff = 0;
    for (int l = 0; l <= kLayers; ++l) {
        const int cin = (l == 0) ? C : ew.w[l - 1];
        const int cout = (l < kLayers) ? ew.w[l] : 1;
        pt.cin[l] = cin;
        pt.cout[l] = cout;
        pt.off[l] = off;
        pt.n[l] = (l < kLayers) ? kTaps * cin * cout + cout : cin + 1;
        pt.split[l] = (l == 0) ? n1split : (l < kLayers) ? nsplit : hsplit;
        pt.poff[l] = poff;
        off += pt.n[l];
        poff += (long long)pt.split[l] * pt.n[l];
    }
    pt.total = off;
    return pt;
}

long long partial_floats(const ParamTable& pt) {
    return pt.poff[kLayers] + (long long)pt.split[kLayers] * pt.n[kLayers];
}

// Canonical (OIHW per layer) <-> internal (tap-major W[t][ci][co]) maps.
void canon_to_internal(const float* src, float* dst, const ParamTable& pt) {
    int co_off = 0;
    for (int l = 0; l <= kLayers; ++l) {
        const int cin = pt.cin[l], cout = pt.cout[l];
        const float* s = src + co_off;
        float* d = dst + pt.off[l];
        if (l < kLayers) {
            for (int co = 0; co < cout; ++co)
                for (int ci = 0; ci < cin; ++ci)
                    for (int t = 0; t < kTaps; ++t) d[(t * cin + ci) * cout + co] = s[(co * cin + ci) * kTaps + t];
            std::memcpy(d + kTaps * cin * cout, s + kTaps * cin * cout, sizeof(float) * cout);
        } else {
            std::memcpy(d, s, sizeof(float) * pt.n[l]);
        }
        co_off += pt.n[l];
    }
}

void internal_to_canon(const float* src, float* dst, const ParamTable& pt) {
    int co_off = 0;
    for (int l = 0; l <= kLayers; ++l) {
        const int cin = pt.cin[l], cout = pt.cout[l];
        const float* s = src + pt.off[l];
        float* d = dst + co_off;
        if (l < kLayers) {
            for (int co = 0; co < cout; ++co)
                for (int ci = 0; ci < cin; ++ci)
                    for (int t = 0; t < kTaps; ++t) d[(co * cin + ci) * kTaps + t] = s[(t * cin + ci) * cout + co];
            std::memcpy(d + kTaps * cin * cout, s + kTaps * cin * cout, sizeof(float) * cout);
        } else {
            std::memcpy(d, s, sizeof(float) * pt.n[l]);
        }
        co_off += pt.n[l];
    }
}

// Workspace carve-out of one run.
struct Plan {
    int H, W, C, Hc, Wc, P, bf;
    int quad, exact;          // 2x2-block downsampling; separate "Exact" target images
    int hu, wu, hl, wl;       // training image shapes of pairs 0-1 and 2-3
    int n1split, nsplit, hsplit, vblk, mmblk, max_trace;
    ParamTable pt;
    size_t o_misc, o_xs, o_ds[4], o_tg[4], o_net[3], net_bytes;
    size_t n_state, n_theta, n_pack32, n_pack16, n_trace, n_img;
    size_t o_act, o_mbits, o_dlt, o_part, o_lpart, o_vpart, bytes;
    size_t act_elems, dlt_elems;
    // offsets inside one network's block
    size_t s_state, s_theta, s_m, s_v, s_g, s_fwd, s_bwd, s_fwd16, s_bwd16, s_trace, s_S, s_yb, s_y;
    // widths other than 64 throughout (generic kernels): per-layer widths,
    // padded input channels of the packed forward operands, packed operand
    // offsets inside a network's block (bytes), stash offsets (elements)
    int gen;
    Widths ew;
    int maxw;
    int cipad[kLayers];
    size_t g_fwd[kLayers], g_bwd[kLayers];
    size_t g_act[kLayers];
};

n2f_status check_cfg(const n2f_config* cfg) {
    if (!cfg) return fail(N2F_EINVAL, "config is NULL");
    if (cfg->n_layers != kLayers) return fail(N2F_EINVAL, "only 8 layers are supported");
    const Widths ew = eff_widths(cfg);
    for (int l = 0; l < kLayers; ++l)
        if (ew.w[l] < 16 || ew.w[l] > 256 || ew.w[l] % 16)
            return fail(N2F_EINVAL, "layer widths must be multiples of 16 from 16 to 256");
    if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
        !(cfg->eps > 0.f))
        return fail(N2F_EINVAL, "bad Adam hyper-parameters");
    if (cfg->patience < 1 || cfg->max_epochs < 1 || cfg->fixed_epochs < 0)
        return fail(N2F_EINVAL, "patience and max_epochs must be >= 1, fixed_epochs >= 0");
    if (cfg->precision != N2F_FP32 && cfg->precision != N2F_BF16) return fail(N2F_EINVAL, "unknown precision");
    if (cfg->downsample != N2F_DS_CHECKERBOARD && cfg->downsample != N2F_DS_QUAD)
        return fail(N2F_EINVAL, "unknown downsample");
    if (cfg->exact_targets != 0 && cfg->exact_targets != 1) return fail(N2F_EINVAL, "exact_targets must be 0 or 1");
    if (cfg->wgrad_splits < 0 || cfg->wgrad_splits > kMaxSplit)
        return fail(N2F_EINVAL, "wgrad_splits must be 0 (default) or 1.." + std::to_string(kMaxSplit));
    int seen[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
        if (cfg->pair_order[i] < 0 || cfg->pair_order[i] > 3 || seen[cfg->pair_order[i]]++)
            return fail(N2F_EINVAL, "pair_order must be a permutation of 0..3");
    }
    return N2F_OK;
}

n2f_status make_plan(int H, int W, int C, const n2f_config* cfg, Plan* p) {
    n2f_status s = check_cfg(cfg);
    if (s != N2F_OK) return s;
    if (H < 2 || W < 2 || C < 1 || C > 3) return fail(N2F_EINVAL, "need H, W >= 2 and 1 <= C <= 3");
    if ((long long)H * W > (1LL << 28)) return fail(N2F_EINVAL, "image too large");
    Plan q{};
    q.H = H;
    q.W = W;
    q.C = C;
    q.bf = cfg->precision == N2F_BF16;
    q.quad = cfg->downsample == N2F_DS_QUAD;
    q.exact = cfg->exact_targets;
    q.Hc = H & ~1;
    q.Wc = W & ~1;
    if (q.quad) {
        q.hu = q.hl = q.Hc / 2;
        q.wu = q.wl = q.Wc / 2;
    } else {
        q.hu = q.Hc;
        q.wu = q.Wc / 2;
        q.hl = q.Hc / 2;
        q.wl = q.Wc;
    }
    q.P = q.hu * q.wu;
    q.ew = eff_widths(cfg);
    q.gen = !is_default_width(q.ew);
    q.maxw = 0;
    for (int l = 0; l < kLayers; ++l) q.maxw = std::max(q.maxw, q.ew.w[l]);
    const long long HW = (long long)H * W;
    if (q.gen) {
        // generic kernels: one split count for every weight gradient (up to
        // 64 tiles' worth of partial rows), one head block per 128 pixels
        auto tiles = [](int h, int w) { return ((w + 15) / 16) * ((h + 15) / 16); };
        q.nsplit = std::max(1, std::min(64, std::max(tiles(q.hu, q.wu), tiles(q.hl, q.wl))));
        q.n1split = q.nsplit;
        q.hsplit = head_splits(q.P);
        q.vblk = head_splits(HW);
    } else {
        q.nsplit = std::max(wgrad_splits(q.hu, q.wu, q.bf, cfg->wgrad_splits),
                            wgrad_splits(q.hl, q.wl, q.bf, cfg->wgrad_splits));
        q.n1split = (int)std::max(1LL, std::min((long long)kMaxSplit, ((long long)q.P + 511) / 512));
        // BF16: the head runs in the last forward convolution's epilogue, one
        // partial row per block of its grid (the larger of the two pair shapes)
        q.hsplit = q.bf ? std::max(head_fused_blocks(q.hu, q.wu), head_fused_blocks(q.hl, q.wl)) : head_splits(q.P);
        q.vblk = (int)std::max(1LL, std::min((HW + 255) / 256, 1024LL));
    }
    q.mmblk = (int)std::max(1LL, std::min((HW * C + 4095) / 4096, 1024LL));
    q.max_trace = std::max(cfg->max_epochs, cfg->fixed_epochs) + 1;
    q.pt = make_table(C, q.ew, q.n1split, q.nsplit, q.hsplit);

    size_t o = 0;
    q.o_misc = o;
    o += align_up(4096 + sizeof(float) * 2 * 1024);
    q.o_xs = o;
    o += align_up(sizeof(float) * HW * C);
    for (int i = 0; i < 4; ++i) {
        q.o_ds[i] = o;
        o += align_up(sizeof(float) * (size_t)q.P * C);
    }
    for (int i = 0; i < 4; ++i) {
        q.o_tg[i] = o;
        if (q.exact) o += align_up(sizeof(float) * (size_t)q.P * C);
    }
    // one network's block
    size_t n = 0;
    q.s_state = n;
    n += align_up(sizeof(DevState));
    const size_t tb = align_up(sizeof(float) * q.pt.total);
    q.s_theta = n;
    n += tb;
    q.s_m = n;
    n += tb;
    q.s_v = n;
    n += tb;
    q.s_g = n;
    n += tb;
    const size_t pk = q.gen ? 0 : (size_t)(kLayers - 1) * kPackN;
    q.s_fwd = n;
    n += q.bf ? 0 : align_up(sizeof(float) * pk);
    q.s_bwd = n;
    n += q.bf ? 0 : align_up(sizeof(float) * pk);
    q.s_fwd16 = n;
    n += q.bf ? align_up(sizeof(uint16_t) * pk) : 0;
    q.s_bwd16 = n;
    n += q.bf ? align_up(sizeof(uint16_t) * pk) : 0;
    if (q.gen) {
        // packed operands of every layer: FP32 for the first layer (and the
        // FP32 path), BF16 for layers 2..8 of a BF16 run
        for (int l = 0; l < kLayers; ++l) {
            q.cipad[l] = l == 0 ? (C + 15) / 16 * 16 : q.ew.w[l - 1];
            const size_t es_w = (q.bf && l > 0) ? 2 : 4;
            q.g_fwd[l] = n;
            n += align_up(es_w * kTaps * q.cipad[l] * q.ew.w[l]);
            q.g_bwd[l] = n;
            if (l > 0) n += align_up(es_w * kTaps * q.ew.w[l] * q.ew.w[l - 1]);
        }
    }
    q.s_trace = n;
    n += align_up(sizeof(double) * q.max_trace);
    q.s_S = n;
    n += align_up(sizeof(float) * HW);
    q.s_yb = n;
    n += align_up(sizeof(float) * HW);
    q.s_y = n;
    n += align_up(sizeof(float) * HW);
    q.net_bytes = n;
    for (int k = 0; k < C; ++k) {
        q.o_net[k] = o;
        o += n;
    }
    const size_t es = q.bf ? 2 : 4;
    if (q.gen) {
        // training stash: layer l's activation at P * (w_0 + .. + w_{l-1});
        // validation ping-pong: two buffers of HW x max width, aliased
        size_t acc = 0;
        for (int l = 0; l < kLayers; ++l) {
            q.g_act[l] = acc;
            acc += (size_t)q.P * q.ew.w[l];
        }
        q.act_elems = std::max<size_t>(acc, (size_t)2 * HW * q.maxw);
        q.dlt_elems = (size_t)q.P * q.maxw;
    } else {
        q.act_elems = (size_t)std::max<long long>(8LL * q.P, 2LL * HW) * kWidth;
        q.dlt_elems = (size_t)q.P * kWidth;
    }
    q.o_act = o;
    o += align_up(es * q.act_elems);
    q.o_mbits = o;      // BF16: ReLU bit masks of stashed layers 0..6, 8 bytes per pixel
    if (q.bf && !q.gen) o += align_up((size_t)(kLayers - 1) * q.P * 8);
    q.o_dlt = o;
    o += 2 * align_up(es * q.dlt_elems);
    q.o_part = o;
    o += align_up(sizeof(float) * partial_floats(q.pt));
    q.o_lpart = o;
    o += align_up(sizeof(double) * kMaxHeadSplit);
    q.o_vpart = o;
    o += align_up(sizeof(double) * 1024);
    q.bytes = o;
    *p = q;
    return N2F_OK;
}

// Kernel-class timing with HIP events on the launch stream (see n2f.h).  A
// record brackets a run of consecutive launches of one class, so the two
// event markers cost once per run rather than once per kernel.
struct ProfRec {
    int cls;
    long long launches, npix;
    hipEvent_t a, b;
};
struct Profiler {
    bool on = false;
    bool capturing = false;
    int every = 1;             // time the launches of one epoch in `every`
    long long epochs = 0;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
} g_prof;

hipEvent_t prof_event() {
    if (g_prof.used < g_prof.pool.size()) return g_prof.pool[g_prof.used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
    g_prof.used++;
    return e;
}

// f() enqueues `launches` kernels of class cls, each over npix pixels.
template <class F>
hipError_t timed(int cls, int launches, long long npix, hipStream_t s, F&& f) {
    if (!g_prof.on || g_prof.capturing) return f();
    hipEvent_t a = prof_event(), b = prof_event();
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    g_prof.recs.push_back({cls, launches, (long long)launches * npix, a, b});
    return e;
}

}  // namespace

struct n2f_run {
    Plan pl;
    n2f_config cfg;
    hipStream_t stream;
    char* ws;
    bool constant;
    const float* in_keep;  // only for constant images (copied at create)
    float lo, hi;
    // device pointers
    float* lohi;
    float* mmpart;
    unsigned* mmcnt;
    int* nonfinite;
    float* xs;
    float* ds[4];
    float* tg[4];      // target image of pair p: ds of its partner, or the "Exact" targets
    bool clean_set;    // exact-target runs: targets built by n2f_run_set_clean
    struct Net {
        DevState* st;
        float *theta, *m, *v, *g, *fwd, *bwd;
        uint16_t *fwd16, *bwd16;
        double* trace;
        float *S, *yb, *y;
        char* base;   // the network's workspace block (generic packed operands)
    } net[3];
    char* act;
    char* mbits;       // BF16 ReLU bit masks of the stashed training layers
    char* dlt[2];
    float* part;
    double* lpart;
    double* vpart;
    bool host_done[3];
    int host_epochs[3];
    hipStream_t cap_stream;          // private stream used only to record graphs
    hipGraph_t graph[3];
    hipGraphExec_t graph_exec[3];    // one captured epoch per network
};

namespace {

template <typename T>
T* at(char* base, size_t off) {
    return reinterpret_cast<T*>(base + off);
}

n2f_status check_run(n2f_run* r, int net) {
    if (!r) return fail(N2F_EINVAL, "run is NULL");
    if (r->constant) return fail(N2F_ESTATE, "constant image: nothing to train");
    if (net < 0 || net >= r->pl.C) return fail(N2F_EINVAL, "network index out of range");
    return N2F_OK;
}

// Training calls of an exact-target run need its targets first.
n2f_status check_targets(n2f_run* r) {
    if (r->pl.exact && !r->clean_set) return fail(N2F_ESTATE, "exact-target run: call n2f_run_set_clean first");
    return N2F_OK;
}

void* act_layer(n2f_run* r, int i, size_t npix) {
    const size_t es = r->pl.bf ? 2 : 4;
    return r->act + es * (size_t)i * npix * kWidth;
}

// ReLU bit mask of stashed training layer i (BF16 runs, i < 7), else NULL.
uint16_t* mask_layer(n2f_run* r, int i, size_t npix) {
    if (!r->pl.bf || i >= kLayers - 1) return nullptr;
    return reinterpret_cast<uint16_t*>(r->mbits) + (size_t)i * npix * 4;
}

// Pair p trains image p towards image kPartner[p] (or its exact target).
constexpr int kPartner[4] = {1, 0, 3, 2};

// Images and shapes of training pair `pair`.
void pair_io(n2f_run* r, int pair, const float** in, const float** tgt, int* h, int* w) {
    *in = r->ds[pair];
    *tgt = r->tg[pair];
    if (pair < 2) {
        *h = r->pl.hu;
        *w = r->pl.wu;
    } else {
        *h = r->pl.hl;
        *w = r->pl.wl;
    }
}

// Packed convolution operands of network k from its parameters (after
// creation, state loads and every Adam step).
hipError_t pack_net(n2f_run* r, int k, hipStream_t s, const DevState* st = nullptr) {
    const Plan& pl = r->pl;
    n2f_run::Net& N = r->net[k];
    if (!pl.gen) return launch_pack(N.theta, pl.pt, N.fwd, N.bwd, N.fwd16, N.bwd16, s);
    for (int l = 0; l < kLayers; ++l) {
        const bool wf = !pl.bf || l == 0;   // FP32 weights: the FP32 path and every first layer
        hipError_t e = launch_gpack(N.theta, pl.pt.off[l], pl.pt.cin[l], pl.pt.cout[l], pl.cipad[l],
                                    N.base + pl.g_fwd[l], l > 0 ? N.base + pl.g_bwd[l] : nullptr, wf, st, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One training step of a network of other widths than 64 (generic kernels):
// the same sequence as the 64-wide step, layer by layer.
n2f_status enqueue_train_step_generic(n2f_run* r, int k, int pair) {
    const Plan& pl = r->pl;
    n2f_run::Net& N = r->net[k];
    const float *in, *tgt;
    int h, w;
    pair_io(r, pair, &in, &tgt, &h, &w);
    const long long npix = (long long)h * w;
    const int bf = pl.bf;
    const ParamTable& pt = pl.pt;
    hipStream_t s = r->stream;
    const size_t es = bf ? 2 : 4;
    auto act = [&](int l) -> void* { return r->act + es * pl.g_act[l]; };   // stash: a_{l+1}
    auto Bl = [&](int l) { return N.theta + pt.off[l] + kTaps * pt.cin[l] * pt.cout[l]; };
    auto fwdpk = [&](int l) -> const void* { return N.base + pl.g_fwd[l]; };
    auto bwdpk = [&](int l) -> const void* { return N.base + pl.g_bwd[l]; };
    N2F_HIP(launch_gconv(in, pl.C, true, fwdpk(0), true, pl.cipad[0], Bl(0), nullptr, act(0), pt.cout[0], 0, bf, h,
                         w, N.st, s));
    for (int l = 1; l < kLayers; ++l)
        N2F_HIP(launch_gconv(act(l - 1), pt.cin[l], false, fwdpk(l), !bf, pl.cipad[l], Bl(l), nullptr, act(l),
                             pt.cout[l], 0, bf, h, w, N.st, s));
    const float* w9 = N.theta + pt.off[kLayers];
    N2F_HIP(launch_ghead(act(kLayers - 1), pt.cin[kLayers], tgt, pl.C, k, w9, r->dlt[0], nullptr,
                         r->part + pt.poff[kLayers], r->lpart, pt.split[kLayers], 1, bf, npix, N.st, s));
    int cur = 0;
    for (int l = kLayers - 1; l >= 1; --l) {
        N2F_HIP(launch_gwgrad(act(l - 1), pt.cin[l], false, r->dlt[cur], pt.cout[l], r->part + pt.poff[l],
                              pt.split[l], bf, h, w, N.st, s));
        N2F_HIP(launch_gconv(r->dlt[cur], pt.cout[l], false, bwdpk(l), !bf, pt.cout[l], nullptr, act(l - 1),
                             r->dlt[1 - cur], pt.cin[l], 1, bf, h, w, N.st, s));
        cur = 1 - cur;
    }
    N2F_HIP(launch_gwgrad(in, pl.C, true, r->dlt[cur], pt.cout[0], r->part + pt.poff[0], pt.split[0], bf, h, w,
                          N.st, s));
    N2F_HIP(launch_gadam(N.theta, N.m, N.v, N.g, r->part, pt, r->cfg.lr, r->cfg.beta1, r->cfg.beta2, r->cfg.eps,
                         r->lpart, pt.split[kLayers], npix, N.st, s));
    N2F_HIP(pack_net(r, k, s, N.st));
    return N2F_OK;
}

// Validation of a network of other widths than 64: full-image forward through
// two ping-pong buffers, the head with the squared-error partials, then the
// stopping decision and the running output sum.
n2f_status enqueue_validate_generic(n2f_run* r, int k) {
    const Plan& pl = r->pl;
    n2f_run::Net& N = r->net[k];
    const ParamTable& pt = pl.pt;
    const int bf = pl.bf;
    const long long HW = (long long)pl.H * pl.W;
    hipStream_t s = r->stream;
    const size_t es = bf ? 2 : 4;
    auto vbuf = [&](int b) -> void* { return r->act + es * (size_t)b * HW * pl.maxw; };
    auto Bl = [&](int l) { return N.theta + pt.off[l] + kTaps * pt.cin[l] * pt.cout[l]; };
    auto fwdpk = [&](int l) -> const void* { return N.base + pl.g_fwd[l]; };
    N2F_HIP(launch_gconv(r->xs, pl.C, true, fwdpk(0), true, pl.cipad[0], Bl(0), nullptr, vbuf(0), pt.cout[0], 0, bf,
                         pl.H, pl.W, N.st, s));
    for (int l = 1; l < kLayers; ++l)
        N2F_HIP(launch_gconv(vbuf((l - 1) & 1), pt.cin[l], false, fwdpk(l), !bf, pl.cipad[l], Bl(l), nullptr,
                             vbuf(l & 1), pt.cout[l], 0, bf, pl.H, pl.W, N.st, s));
    const float* w9 = N.theta + pt.off[kLayers];
    N2F_HIP(launch_ghead(vbuf((kLayers - 1) & 1), pt.cin[kLayers], r->xs, pl.C, k, w9, nullptr, N.y, nullptr, r->vpart,
                         pl.vblk, 0, bf, HW, N.st, s));
    N2F_HIP(launch_decide(r->vpart, pl.vblk, HW, N.st, N.trace, s));
    N2F_HIP(launch_accumulate(N.y, N.S, N.yb, HW, N.st, s));
    return N2F_OK;
}

n2f_status enqueue_train_step(n2f_run* r, int k, int pair) {
    if (r->pl.gen) return enqueue_train_step_generic(r, k, pair);
    const Plan& pl = r->pl;
    n2f_run::Net& N = r->net[k];
    const float *in, *tgt;
    int h, w;
    pair_io(r, pair, &in, &tgt, &h, &w);
    const size_t npix = (size_t)h * w;
    const int bf = pl.bf;
    const ParamTable& pt = pl.pt;
    hipStream_t s = r->stream;
    auto Wl = [&](int l) { return N.theta + pt.off[l]; };                       // layer l, 0-based
    auto Bl = [&](int l) { return N.theta + pt.off[l] + kTaps * pt.cin[l] * kWidth; };
    auto fwdpk = [&](int l) -> const void* {
        return bf ? (const void*)(N.fwd16 + (size_t)(l - 1) * kPackN) : (const void*)(N.fwd + (size_t)(l - 1) * kPackN);
    };
    auto bwdpk = [&](int l) -> const void* {
        return bf ? (const void*)(N.bwd16 + (size_t)(l - 1) * kPackN) : (const void*)(N.bwd + (size_t)(l - 1) * kPackN);
    };
    // forward with stash: act layer i holds a_{i+1}; BF16 fuses the head
    // into the last layer, whose a8 is then never stored
    // BF16 with one channel also computes the first layer inside the layer-2
    // forward (a1 and its mask are still stored for the backward pass)
    const int nplain = bf ? kLayers - 2 : kLayers - 1;
    const bool first_fused = bf && pl.C == 1;
    if (first_fused) {
        ConvFirst cf{in, Wl(0), Bl(0), (uint16_t*)act_layer(r, 0, npix), mask_layer(r, 0, npix)};
        N2F_HIP(launch_conv_fwd_first(cf, fwdpk(1), Bl(1), act_layer(r, 1, npix), mask_layer(r, 1, npix), h, w, N.st,
                                      s));
    } else {
        N2F_HIP(launch_conv1(in, pl.C, Wl(0), Bl(0), act_layer(r, 0, npix), mask_layer(r, 0, npix), bf, h, w, N.st,
                             s));
    }
    const int lfirst = first_fused ? 2 : 1;
    N2F_HIP(timed(N2F_K_CONV_FWD, nplain - lfirst + 1, (long long)npix, s, [&]() -> hipError_t {
        for (int l = lfirst; l <= nplain; ++l) {
            hipError_t e = launch_conv_fwd(act_layer(r, l - 1, npix), fwdpk(l), Bl(l), act_layer(r, l, npix),
                                           mask_layer(r, l, npix), bf, h, w, N.st, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }));
    // head, BCE gradient
    const float* w9 = N.theta + pt.off[kLayers];
    if (bf) {
        ConvHead hd{w9, tgt, r->part + pt.poff[kLayers], r->lpart, nullptr, N.st, pl.C, k, 1.0f / (float)npix};
        N2F_HIP(launch_conv_fwd_head(act_layer(r, kLayers - 2, npix), fwdpk(kLayers - 1), Bl(kLayers - 1), r->dlt[0],
                                     hd, pt.split[kLayers], h, w, N.st, s));
    } else {
        N2F_HIP(launch_head_train(act_layer(r, kLayers - 1, npix), tgt, pl.C, k, w9, w9 + kWidth, r->dlt[0],
                                  r->part + pt.poff[kLayers], r->lpart, pt.split[kLayers], bf, (long long)npix, N.st,
                                  s));
    }
    // backward: layer l (0-based 7..1) takes delta of its output
    int cur = 0;
    N2F_HIP(timed(N2F_K_BACKWARD, kLayers - 1, (long long)npix, s, [&]() -> hipError_t {
        for (int l = kLayers - 1; l >= 1; --l) {
            hipError_t e = launch_wgrad(act_layer(r, l - 1, npix), r->dlt[cur], r->part + pt.poff[l], pt.split[l], bf,
                                        h, w, N.st, s);
            if (e != hipSuccess) return e;
            const void* mask = bf ? (const void*)mask_layer(r, l - 1, npix) : act_layer(r, l - 1, npix);
            e = launch_conv_bwd(r->dlt[cur], bwdpk(l), mask, r->dlt[1 - cur], bf, h, w, N.st, s);
            if (e != hipSuccess) return e;
            cur = 1 - cur;
        }
        return hipSuccess;
    }));
    N2F_HIP(launch_wgrad1(in, pl.C, r->dlt[cur], r->part + pt.poff[0], pt.split[0], bf, h, w, N.st, s));
    N2F_HIP(timed(N2F_K_ADAM, 1, (long long)npix, s, [&] {
        return launch_adam(N.theta, N.m, N.v, N.g, r->part, nullptr, pt, r->cfg.lr, r->cfg.beta1, r->cfg.beta2,
                           r->cfg.eps, N.fwd, N.bwd, N.fwd16, N.bwd16, r->lpart, pt.split[kLayers], (long long)npix,
                           N.st, s);
    }));
    return N2F_OK;
}

n2f_status enqueue_validate(n2f_run* r, int k) {
    if (r->pl.gen) return enqueue_validate_generic(r, k);
    const Plan& pl = r->pl;
    n2f_run::Net& N = r->net[k];
    const ParamTable& pt = pl.pt;
    const int bf = pl.bf;
    const size_t npix = (size_t)pl.H * pl.W;
    hipStream_t s = r->stream;
    auto buf = [&](int i) { return act_layer(r, i & 1, npix); };
    auto Bl = [&](int l) { return N.theta + pt.off[l] + kTaps * pt.cin[l] * kWidth; };
    auto pk = [&](int l) -> const void* {
        return bf ? (const void*)(N.fwd16 + (size_t)(l - 1) * kPackN) : (const void*)(N.fwd + (size_t)(l - 1) * kPackN);
    };
    // BF16 fuses the head into the last layer (see enqueue_train_step)
    const int nplain = bf ? kLayers - 2 : kLayers - 1;
    const bool first_fused = bf && pl.C == 1;   // as in enqueue_train_step; a1 is not stored here
    if (first_fused) {
        ConvFirst cf{r->xs, N.theta + pt.off[0], Bl(0), nullptr, nullptr};
        N2F_HIP(launch_conv_fwd_first(cf, pk(1), Bl(1), buf(1), nullptr, pl.H, pl.W, N.st, s));
    } else {
        N2F_HIP(launch_conv1(r->xs, pl.C, N.theta + pt.off[0], Bl(0), buf(0), nullptr, bf, pl.H, pl.W, N.st, s));
    }
    const int lfirst = first_fused ? 2 : 1;
    N2F_HIP(timed(N2F_K_CONV_FWD, nplain - lfirst + 1, (long long)npix, s, [&]() -> hipError_t {
        for (int l = lfirst; l <= nplain; ++l) {
            hipError_t e = launch_conv_fwd(buf(l - 1), pk(l), Bl(l), buf(l), nullptr, bf, pl.H, pl.W, N.st, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }));
    const float* w9 = N.theta + pt.off[kLayers];
    if (bf) {
        ConvHead hd{w9, r->xs, nullptr, r->vpart, N.y, N.st, pl.C, k, 0.f};
        N2F_HIP(launch_conv_fwd_val(buf(kLayers - 2), pk(kLayers - 1), Bl(kLayers - 1), hd, pl.H, pl.W, N.st, N.trace,
                                    s));
    } else {
        N2F_HIP(launch_head_val(buf(kLayers - 1), r->xs, pl.C, k, w9, w9 + kWidth, N.y, r->vpart, pl.vblk, bf,
                                (long long)npix, N.st, N.trace, s));
    }
    N2F_HIP(launch_accumulate(N.y, N.S, N.yb, (long long)npix, N.st, s));
    return N2F_OK;
}

n2f_status read_state(n2f_run* r, int k, DevState* out) {
    N2F_HIP(hipMemcpyAsync(out, r->net[k].st, sizeof(DevState), hipMemcpyDeviceToHost, r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    return N2F_OK;
}

n2f_status enqueue_epoch(n2f_run* r, int k) {
    for (int i = 0; i < 4; ++i) {
        n2f_status s = enqueue_train_step(r, k, r->cfg.pair_order[i]);
        if (s != N2F_OK) return s;
    }
    return enqueue_validate(r, k);
}

// Record one epoch of network k (four steps and the validation) as a graph.
// Every kernel reads its state from device memory and returns at once when
// the network is finished, so the same graph is replayed every epoch.
n2f_status capture_epoch(n2f_run* r, int k) {
    if (!r->cap_stream) N2F_HIP(hipStreamCreateWithFlags(&r->cap_stream, hipStreamNonBlocking));
    hipStream_t user = r->stream;
    r->stream = r->cap_stream;
    g_prof.capturing = true;
    hipError_t e = hipStreamBeginCapture(r->cap_stream, hipStreamCaptureModeRelaxed);
    n2f_status s = N2F_OK;
    if (e == hipSuccess) s = enqueue_epoch(r, k);
    hipGraph_t g = nullptr;
    hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(r->cap_stream, &g) : e;
    g_prof.capturing = false;
    r->stream = user;
    if (e != hipSuccess || e2 != hipSuccess || s != N2F_OK) {
        if (g) (void)hipGraphDestroy(g);
        if (s != N2F_OK) return s;
        return fail(N2F_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(N2F_EDEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(e));
    }
    r->graph[k] = g;
    r->graph_exec[k] = ex;
    return N2F_OK;
}

}  // namespace

extern "C" {

void n2f_config_default(n2f_config* cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_layers = kLayers;
    cfg->width = kWidth;
    cfg->lr = 1e-3f;
    cfg->beta1 = 0.9;
    cfg->beta2 = 0.999;
    cfg->eps = 1e-8f;
    cfg->patience = 100;
    cfg->max_epochs = 2000;
    cfg->fixed_epochs = 0;
    for (int i = 0; i < 4; ++i) cfg->pair_order[i] = i;
    cfg->precision = N2F_FP32;
    cfg->init_seed = 0;
    cfg->use_graph = 1;
    cfg->downsample = N2F_DS_CHECKERBOARD;
    cfg->exact_targets = 0;
}

const char* n2f_last_error(void) { return g_err.c_str(); }

}  // extern "C"

void n2f::set_last_error(const char* msg) { g_err = msg; }

extern "C" {

n2f_status n2f_param_count(int C, const n2f_config* cfg, size_t* count) {
    n2f_status s = check_cfg(cfg);
    if (s != N2F_OK) return s;
    if (C < 1 || C > 3 || !count) return fail(N2F_EINVAL, "need 1 <= C <= 3 and a non-NULL count");
    *count = (size_t)make_table(C, eff_widths(cfg), 1, 1, 1).total;
    return N2F_OK;
}

n2f_status n2f_init_params(int C, const n2f_config* cfg, unsigned long long seed, float* theta) {
    size_t np;
    n2f_status s = n2f_param_count(C, cfg, &np);
    if (s != N2F_OK) return s;
    if (!theta) return fail(N2F_EINVAL, "theta is NULL");
    const auto L = canon_layers(C, eff_widths(cfg));
    for (int k = 0; k < C; ++k) {
        size_t i = 0;
        for (const CanonLayer& cl : L) {
            const int fan_in = cl.cin * cl.taps;
            const double bound = 1.0 / std::sqrt((double)fan_in);
            const size_t nl = (size_t)cl.cout * cl.cin * cl.taps + cl.cout;
            for (size_t j = 0; j < nl; ++j, ++i) {
                const unsigned long long z = splitmix64(seed, (unsigned long long)k * np + i);
                const double u = (double)(z >> 11) * 0x1.0p-53;
                theta[(size_t)k * np + i] = (float)((2.0 * u - 1.0) * bound);
            }
        }
    }
    return N2F_OK;
}

n2f_status n2f_workspace_bytes(int H, int W, int C, const n2f_config* cfg, size_t* bytes) {
    if (!bytes) return fail(N2F_EINVAL, "bytes is NULL");
    Plan p;
    n2f_status s = make_plan(H, W, C, cfg, &p);
    if (s != N2F_OK) return s;
    *bytes = p.bytes;
    return N2F_OK;
}

n2f_status n2f_run_create(n2f_run** out, const float* d_in, int H, int W, int C, const n2f_config* cfg,
                          void* d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!out) return fail(N2F_EINVAL, "run pointer is NULL");
    *out = nullptr;
    if (!d_in || !d_ws) return fail(N2F_EINVAL, "input or workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(N2F_EINVAL, "workspace must be 256-byte aligned");
    Plan pl;
    n2f_status s = make_plan(H, W, C, cfg, &pl);
    if (s != N2F_OK) return s;
    if (ws_bytes < pl.bytes)
        return fail(N2F_ENOMEM, "workspace too small: need " + std::to_string(pl.bytes) + " bytes");
    n2f_run* r = new (std::nothrow) n2f_run();
    if (!r) return fail(N2F_ENOMEM, "host allocation failed");
    r->pl = pl;
    r->cfg = *cfg;
    r->stream = stream;
    r->ws = static_cast<char*>(d_ws);
    r->constant = false;
    r->in_keep = nullptr;
    r->cap_stream = nullptr;
    for (int k = 0; k < 3; ++k) {
        r->graph[k] = nullptr;
        r->graph_exec[k] = nullptr;
    }
    char* b = r->ws;
    char* misc = b + pl.o_misc;
    r->lohi = at<float>(misc, 0);
    r->mmcnt = at<unsigned>(misc, 64);
    r->nonfinite = at<int>(misc, 128);
    r->mmpart = at<float>(misc, 4096);
    r->xs = at<float>(b, pl.o_xs);
    for (int i = 0; i < 4; ++i) r->ds[i] = at<float>(b, pl.o_ds[i]);
    for (int i = 0; i < 4; ++i) r->tg[i] = pl.exact ? at<float>(b, pl.o_tg[i]) : r->ds[kPartner[i]];
    r->clean_set = false;
    for (int k = 0; k < C; ++k) {
        char* nb = b + pl.o_net[k];
        n2f_run::Net& N = r->net[k];
        N.st = at<DevState>(nb, pl.s_state);
        N.theta = at<float>(nb, pl.s_theta);
        N.m = at<float>(nb, pl.s_m);
        N.v = at<float>(nb, pl.s_v);
        N.g = at<float>(nb, pl.s_g);
        N.fwd = pl.bf ? nullptr : at<float>(nb, pl.s_fwd);
        N.bwd = pl.bf ? nullptr : at<float>(nb, pl.s_bwd);
        N.fwd16 = pl.bf ? at<uint16_t>(nb, pl.s_fwd16) : nullptr;
        N.bwd16 = pl.bf ? at<uint16_t>(nb, pl.s_bwd16) : nullptr;
        N.trace = at<double>(nb, pl.s_trace);
        N.S = at<float>(nb, pl.s_S);
        N.yb = at<float>(nb, pl.s_yb);
        N.y = at<float>(nb, pl.s_y);
        N.base = nb;
        r->host_done[k] = false;
        r->host_epochs[k] = 0;
    }
    r->act = b + pl.o_act;
    r->mbits = b + pl.o_mbits;
    const size_t es = pl.bf ? 2 : 4;
    r->dlt[0] = b + pl.o_dlt;
    r->dlt[1] = b + pl.o_dlt + align_up(es * pl.dlt_elems);
    r->part = at<float>(b, pl.o_part);
    r->lpart = at<double>(b, pl.o_lpart);
    r->vpart = at<double>(b, pl.o_vpart);

    auto bail = [&](n2f_status st) {
        delete r;
        return st;
    };
    hipStream_t sm = stream;
    if (hipMemsetAsync(misc, 0, 4096, sm) != hipSuccess) return bail(fail(N2F_EDEVICE, "memset failed"));
    const long long n = (long long)H * W * C;
    if (launch_minmax(d_in, n, r->mmpart, pl.mmblk, r->mmcnt, r->lohi, r->nonfinite, sm) != hipSuccess)
        return bail(fail(N2F_EDEVICE, "minmax launch failed"));
    float lohi[2];
    int nonfin = 0;
    if (hipMemcpyAsync(lohi, r->lohi, sizeof(lohi), hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipMemcpyAsync(&nonfin, r->nonfinite, sizeof(int), hipMemcpyDeviceToHost, sm) != hipSuccess ||
        hipStreamSynchronize(sm) != hipSuccess)
        return bail(fail(N2F_EDEVICE, "reading min/max failed"));
    if (nonfin) return bail(fail(N2F_EINVAL, "input holds NaN or infinite values"));
    r->lo = lohi[0];
    r->hi = lohi[1];
    if (!(lohi[1] > lohi[0])) {
        r->constant = true;
        r->in_keep = d_in;
        // keep a copy of the input inside the workspace (xs has room for it)
        if (hipMemcpyAsync(r->xs, d_in, sizeof(float) * n, hipMemcpyDeviceToDevice, sm) != hipSuccess ||
            hipStreamSynchronize(sm) != hipSuccess)
            return bail(fail(N2F_EDEVICE, "copy failed"));
        *out = r;
        g_err = "constant image";
        return N2F_WCONSTANT;
    }
    if (launch_prepare(d_in, H, W, C, r->lohi, r->xs, r->ds[0], r->ds[1], r->ds[2], r->ds[3], pl.quad, sm) !=
        hipSuccess)
        return bail(fail(N2F_EDEVICE, "prepare launch failed"));
    // initial weights, drawn on the host and copied once
    std::vector<float> th0((size_t)C * pl.pt.total), internal(pl.pt.total);
    n2f_init_params(C, cfg, cfg->init_seed, th0.data());
    for (int k = 0; k < C; ++k) {
        n2f_run::Net& N = r->net[k];
        canon_to_internal(th0.data() + (size_t)k * pl.pt.total, internal.data(), pl.pt);
        if (hipMemcpyAsync(N.theta, internal.data(), sizeof(float) * pl.pt.total, hipMemcpyHostToDevice, sm) !=
                hipSuccess ||
            hipMemsetAsync(N.m, 0, sizeof(float) * pl.pt.total, sm) != hipSuccess ||
            hipMemsetAsync(N.v, 0, sizeof(float) * pl.pt.total, sm) != hipSuccess ||
            hipMemsetAsync(N.g, 0, sizeof(float) * pl.pt.total, sm) != hipSuccess ||
            hipMemsetAsync(N.S, 0, sizeof(float) * H * W, sm) != hipSuccess ||
            hipMemsetAsync(N.yb, 0, sizeof(float) * H * W, sm) != hipSuccess ||
            hipMemsetAsync(N.y, 0, sizeof(float) * H * W, sm) != hipSuccess ||
            launch_init_state(N.st, cfg->patience, cfg->max_epochs, cfg->fixed_epochs, sm) != hipSuccess ||
            pack_net(r, k, sm) != hipSuccess ||
            hipStreamSynchronize(sm) != hipSuccess)  // host buffer must outlive the copy
            return bail(fail(N2F_EDEVICE, "initialising network state failed"));
    }
    *out = r;
    return N2F_OK;
}

n2f_status n2f_run_destroy(n2f_run* r) {
    if (!r) return fail(N2F_EINVAL, "run is NULL");
    for (int k = 0; k < 3; ++k) {
        if (r->graph_exec[k]) (void)hipGraphExecDestroy(r->graph_exec[k]);
        if (r->graph[k]) (void)hipGraphDestroy(r->graph[k]);
    }
    if (r->cap_stream) (void)hipStreamDestroy(r->cap_stream);
    delete r;
    return N2F_OK;
}

n2f_status n2f_train_step(n2f_run* r, int net, int pair) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (pair < 0 || pair > 3) return fail(N2F_EINVAL, "pair must be 0..3");
    if (r->host_done[net]) return fail(N2F_ESTATE, "network already finished");
    s = check_targets(r);
    if (s != N2F_OK) return s;
    return enqueue_train_step(r, net, pair);
}

n2f_status n2f_validate(n2f_run* r, int net, double* v, int* improved, int* done) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (r->host_done[net]) return fail(N2F_ESTATE, "network already finished");
    s = enqueue_validate(r, net);
    if (s != N2F_OK) return s;
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    r->host_done[net] = st.done != 0;
    r->host_epochs[net] = st.epoch;
    if (v) *v = st.last_v;
    if (improved) *improved = st.improved;
    if (done) *done = st.done;
    if (st.nonfinite) return fail(N2F_ENUMERIC, "validation score is not finite");
    return N2F_OK;
}

n2f_status n2f_run_epochs(n2f_run* r, int net, int max_now, int* done) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (max_now < 1) return fail(N2F_EINVAL, "max_epochs_now must be >= 1");
    s = check_targets(r);
    if (s != N2F_OK) return s;
    if (r->cfg.use_graph && !r->graph_exec[net]) {
        s = capture_epoch(r, net);
        if (s != N2F_OK) return s;
    }
    DevState st;
    int ran = 0;
    while (!r->host_done[net] && ran < max_now) {
        // queue a few epochs ahead, then poll the device-side stopping rule
        const int batch = std::min(max_now - ran, 4);
        for (int e = 0; e < batch; ++e) {
            const bool direct = !r->graph_exec[net] || (g_prof.on && (g_prof.epochs++ % g_prof.every) == 0);
            if (direct) {
                s = enqueue_epoch(r, net);
                if (s != N2F_OK) return s;
            } else {
                N2F_HIP(hipGraphLaunch(r->graph_exec[net], r->stream));
            }
        }
        ran += batch;
        s = read_state(r, net, &st);
        if (s != N2F_OK) return s;
        r->host_done[net] = st.done != 0;
        r->host_epochs[net] = st.epoch;
    }
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    if (done) *done = st.done;
    if (st.nonfinite) return fail(N2F_ENUMERIC, "validation score is not finite");
    if (st.capped) return N2F_WCAPPED;
    return N2F_OK;
}

n2f_status n2f_run_launch_epochs(n2f_run* r, int net, int n_epochs) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (n_epochs < 1) return fail(N2F_EINVAL, "n_epochs must be >= 1");
    s = check_targets(r);
    if (s != N2F_OK) return s;
    if (r->host_done[net]) return N2F_OK;
    if (r->cfg.use_graph && !r->graph_exec[net]) {
        s = capture_epoch(r, net);
        if (s != N2F_OK) return s;
    }
    for (int e = 0; e < n_epochs; ++e) {
        if (r->graph_exec[net]) {
            N2F_HIP(hipGraphLaunch(r->graph_exec[net], r->stream));
        } else {
            s = enqueue_epoch(r, net);
            if (s != N2F_OK) return s;
        }
    }
    return N2F_OK;
}

n2f_status n2f_run_poll(n2f_run* r, int net, int* done, int* epochs) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    r->host_done[net] = st.done != 0;
    r->host_epochs[net] = st.epoch;
    if (done) *done = st.done;
    if (epochs) *epochs = st.epoch;
    if (st.nonfinite) return fail(N2F_ENUMERIC, "validation score is not finite");
    if (st.capped) return N2F_WCAPPED;
    return N2F_OK;
}

n2f_status n2f_result(n2f_run* r, float* d_out) {
    if (!r || !d_out) return fail(N2F_EINVAL, "run or output is NULL");
    const Plan& pl = r->pl;
    const long long npix = (long long)pl.H * pl.W;
    if (r->constant) {
        N2F_HIP(hipMemcpyAsync(d_out, r->xs, sizeof(float) * npix * pl.C, hipMemcpyDeviceToDevice, r->stream));
        return N2F_WCONSTANT;
    }
    for (int k = 0; k < pl.C; ++k) {
        n2f_run::Net& N = r->net[k];
        N2F_HIP(launch_finalize(N.y, N.S, N.yb, r->lohi, d_out + (size_t)k * npix, npix, N.st, r->stream));
    }
    return N2F_OK;
}

n2f_status n2f_denoise(const float* d_in, float* d_out, int H, int W, int C, const n2f_config* cfg, void* d_ws,
                       size_t ws_bytes, hipStream_t stream) {
    if (cfg && cfg->exact_targets) return fail(N2F_EINVAL, "exact targets need the clean image: use a run");
    n2f_run* r = nullptr;
    n2f_status s = n2f_run_create(&r, d_in, H, W, C, cfg, d_ws, ws_bytes, stream);
    if (s < 0) return s;
    n2f_status warn = N2F_OK;
    if (s == N2F_OK) {
        const int cap = cfg->fixed_epochs > 0 ? cfg->fixed_epochs : cfg->max_epochs;
        for (int k = 0; k < C; ++k) {
            int done = 0;
            s = n2f_run_epochs(r, k, cap, &done);
            if (s < 0) {
                n2f_run_destroy(r);
                return s;
            }
            if (s == N2F_WCAPPED) warn = N2F_WCAPPED;
        }
    }
    s = n2f_result(r, d_out);
    if (s >= 0 && hipStreamSynchronize(stream) != hipSuccess) s = fail(N2F_EDEVICE, "synchronise failed");
    n2f_run_destroy(r);
    if (s < 0) return s;
    return s == N2F_WCONSTANT ? s : warn;
}

n2f_status n2f_run_set_clean(n2f_run* r, const float* d_clean) {
    if (!r || !d_clean) return fail(N2F_EINVAL, "run or clean image is NULL");
    if (r->constant) return fail(N2F_ESTATE, "constant image: nothing to train");
    if (!r->pl.exact) return fail(N2F_ESTATE, "run was not created with exact_targets");
    const Plan& pl = r->pl;
    hipStream_t sm = r->stream;
    const long long n = (long long)pl.H * pl.W * pl.C;
    // finiteness check with the run's min/max kernel, into spare words of
    // the misc block (the run's own extremes stay untouched)
    char* misc = r->ws + pl.o_misc;
    float* lohi2 = at<float>(misc, 256);
    int nonfin = 0;
    N2F_HIP(launch_minmax(d_clean, n, r->mmpart, pl.mmblk, r->mmcnt, lohi2, r->nonfinite, sm));
    N2F_HIP(hipMemcpyAsync(&nonfin, r->nonfinite, sizeof(int), hipMemcpyDeviceToHost, sm));
    N2F_HIP(hipStreamSynchronize(sm));
    if (nonfin) {
        N2F_HIP(hipMemsetAsync(r->nonfinite, 0, sizeof(int), sm));
        N2F_HIP(hipStreamSynchronize(sm));
        return fail(N2F_EINVAL, "clean image holds NaN or infinite values");
    }
    // the clean downsamples, standardised with the noisy extremes, into the
    // target images (the activation stash holds the unused full image),
    // then the targets in place
    float* scratch = reinterpret_cast<float*>(r->act);
    N2F_HIP(launch_prepare(d_clean, pl.H, pl.W, pl.C, r->lohi, scratch, r->tg[0], r->tg[1], r->tg[2], r->tg[3],
                           pl.quad, sm));
    const float* x[4] = {r->ds[0], r->ds[1], r->ds[2], r->ds[3]};
    N2F_HIP(launch_exact_targets(x, r->tg, (long long)pl.P * pl.C, sm));
    N2F_HIP(hipStreamSynchronize(sm));
    r->clean_set = true;
    return N2F_OK;
}

n2f_status n2f_max_project(const float* d_stack, int n_slices, long long npix, float* d_out, hipStream_t stream) {
    if (!d_stack || !d_out) return fail(N2F_EINVAL, "stack or output is NULL");
    if (n_slices < 1 || npix < 1) return fail(N2F_EINVAL, "need n_slices >= 1 and npix >= 1");
    if (npix > (1LL << 40) / n_slices) return fail(N2F_EINVAL, "stack too large");
    const uintptr_t a = reinterpret_cast<uintptr_t>(d_stack), b = reinterpret_cast<uintptr_t>(d_out);
    if (b < a + sizeof(float) * (uintptr_t)n_slices * (uintptr_t)npix && a < b + sizeof(float) * (uintptr_t)npix)
        return fail(N2F_EINVAL, "output overlaps the stack");
    N2F_HIP(launch_max_project(d_stack, n_slices, npix, d_out, stream));
    return N2F_OK;
}

n2f_status n2f_get_state(n2f_run* r, int net, float* theta, float* m, float* v, long long* t) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    const ParamTable& pt = r->pl.pt;
    n2f_run::Net& N = r->net[net];
    std::vector<float> tmp(pt.total);
    float* dsts[3] = {theta, m, v};
    float* srcs[3] = {N.theta, N.m, N.v};
    for (int i = 0; i < 3; ++i) {
        if (!dsts[i]) continue;
        N2F_HIP(hipMemcpyAsync(tmp.data(), srcs[i], sizeof(float) * pt.total, hipMemcpyDeviceToHost, r->stream));
        N2F_HIP(hipStreamSynchronize(r->stream));
        internal_to_canon(tmp.data(), dsts[i], pt);
    }
    if (t) {
        DevState st;
        s = read_state(r, net, &st);
        if (s != N2F_OK) return s;
        *t = st.t;
    }
    return N2F_OK;
}

n2f_status n2f_set_state(n2f_run* r, int net, const float* theta, const float* m, const float* v, long long t) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (!theta || t < 0) return fail(N2F_EINVAL, "theta is NULL or t < 0");
    const ParamTable& pt = r->pl.pt;
    n2f_run::Net& N = r->net[net];
    std::vector<float> tmp(pt.total);
    const float* srcs[3] = {theta, m, v};
    float* dsts[3] = {N.theta, N.m, N.v};
    for (int i = 0; i < 3; ++i) {
        if (srcs[i]) {
            canon_to_internal(srcs[i], tmp.data(), pt);
            N2F_HIP(hipMemcpyAsync(dsts[i], tmp.data(), sizeof(float) * pt.total, hipMemcpyHostToDevice, r->stream));
            N2F_HIP(hipStreamSynchronize(r->stream));
        } else {
            N2F_HIP(hipMemsetAsync(dsts[i], 0, sizeof(float) * pt.total, r->stream));
        }
    }
    N2F_HIP(pack_net(r, net, r->stream));
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    st.t = t;
    N2F_HIP(hipMemcpyAsync(N.st, &st, sizeof(DevState), hipMemcpyHostToDevice, r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    return N2F_OK;
}

}  // extern "C"

namespace {
// Checkpoint blob: this header, then a copy of the network's workspace block
// (state struct, parameters, moments, packed weights, validation history,
// running output sum, best and last outputs).  The fields below fix that
// block's layout, so a checkpoint loads only into a run that matches them.
struct CkptHeader {
    unsigned long long magic;
    int H, W, C, precision, downsample, exact, max_trace, reserved;
    int widths[kLayers];
    unsigned long long net_bytes;
};
constexpr unsigned long long kCkptMagic = 0x32544b4350463248ULL;   // "H2FPCKT2"

CkptHeader ckpt_header(const n2f_run* r) {
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.H = r->pl.H;
    h.W = r->pl.W;
    h.C = r->pl.C;
    h.precision = r->pl.bf;
    h.downsample = r->pl.quad;
    h.exact = r->pl.exact;
    h.max_trace = r->pl.max_trace;
    for (int l = 0; l < kLayers; ++l) h.widths[l] = r->pl.ew.w[l];
    h.net_bytes = r->pl.net_bytes;
    return h;
}
}  // namespace

extern "C" {

n2f_status n2f_checkpoint_bytes(n2f_run* r, size_t* bytes) {
    if (!r || !bytes) return fail(N2F_EINVAL, "run or bytes is NULL");
    if (r->constant) return fail(N2F_ESTATE, "constant image: nothing to checkpoint");
    *bytes = sizeof(CkptHeader) + r->pl.net_bytes;
    return N2F_OK;
}

n2f_status n2f_save_checkpoint(n2f_run* r, int net, void* buf, size_t bytes) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (!buf || bytes < sizeof(CkptHeader) + r->pl.net_bytes) return fail(N2F_EINVAL, "checkpoint buffer too small");
    const CkptHeader h = ckpt_header(r);
    std::memcpy(buf, &h, sizeof(h));
    N2F_HIP(hipMemcpyAsync(static_cast<char*>(buf) + sizeof(h), r->ws + r->pl.o_net[net], r->pl.net_bytes,
                           hipMemcpyDeviceToHost, r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    return N2F_OK;
}

n2f_status n2f_load_checkpoint(n2f_run* r, int net, const void* buf, size_t bytes) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (!buf || bytes < sizeof(CkptHeader)) return fail(N2F_EINVAL, "checkpoint buffer too small");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    const CkptHeader mine = ckpt_header(r);
    if (h.magic != kCkptMagic) return fail(N2F_EINVAL, "not a checkpoint");
    if (h.H != mine.H || h.W != mine.W || h.C != mine.C || h.precision != mine.precision ||
        h.downsample != mine.downsample || h.exact != mine.exact || h.max_trace != mine.max_trace ||
        std::memcmp(h.widths, mine.widths, sizeof(h.widths)) != 0 || h.net_bytes != mine.net_bytes)
        return fail(N2F_EINVAL, "checkpoint of a different image size or configuration");
    if (bytes < sizeof(h) + h.net_bytes) return fail(N2F_EINVAL, "checkpoint buffer too small");
    N2F_HIP(hipMemcpyAsync(r->ws + r->pl.o_net[net], static_cast<const char*>(buf) + sizeof(h), r->pl.net_bytes,
                           hipMemcpyHostToDevice, r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    r->host_done[net] = st.done != 0;
    r->host_epochs[net] = st.epoch;
    return N2F_OK;
}

n2f_status n2f_get_grad(n2f_run* r, int net, float* g, double* loss) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    const ParamTable& pt = r->pl.pt;
    if (g) {
        std::vector<float> tmp(pt.total);
        N2F_HIP(hipMemcpyAsync(tmp.data(), r->net[net].g, sizeof(float) * pt.total, hipMemcpyDeviceToHost, r->stream));
        N2F_HIP(hipStreamSynchronize(r->stream));
        internal_to_canon(tmp.data(), g, pt);
    }
    if (loss) {
        DevState st;
        s = read_state(r, net, &st);
        if (s != N2F_OK) return s;
        *loss = st.loss;
    }
    return N2F_OK;
}

n2f_status n2f_debug_adam(n2f_run* r, int net, const float* g) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (!g) return fail(N2F_EINVAL, "gradient is NULL");
    if (r->host_done[net]) return fail(N2F_ESTATE, "network already finished");
    if (r->pl.gen) return fail(N2F_EINVAL, "injected-gradient Adam steps are for the 64-wide network only");
    const ParamTable& pt = r->pl.pt;
    n2f_run::Net& N = r->net[net];
    std::vector<float> tmp(pt.total);
    canon_to_internal(g, tmp.data(), pt);
    // stage the injected gradient in the partial-sum buffer (unused between steps)
    N2F_HIP(hipMemcpyAsync(r->part, tmp.data(), sizeof(float) * pt.total, hipMemcpyHostToDevice, r->stream));
    N2F_HIP(launch_adam(N.theta, N.m, N.v, N.g, r->part, r->part, pt, r->cfg.lr, r->cfg.beta1,
                        r->cfg.beta2, r->cfg.eps, N.fwd, N.bwd, N.fwd16, N.bwd16, r->lpart, 0, 1, N.st,
                        r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    return N2F_OK;
}

n2f_status n2f_get_progress(n2f_run* r, int net, int* epoch, int* best_epoch, int* since_best, double* best) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    if (epoch) *epoch = st.epoch;
    if (best_epoch) *best_epoch = st.best_epoch;
    if (since_best) *since_best = st.n_since;
    if (best) *best = st.best;
    return N2F_OK;
}

n2f_status n2f_get_history(n2f_run* r, int net, int n, double* v) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    DevState st;
    s = read_state(r, net, &st);
    if (s != N2F_OK) return s;
    if (n < 0 || n > st.epoch || (n > 0 && !v)) return fail(N2F_EINVAL, "n exceeds the epochs run");
    if (n == 0) return N2F_OK;
    N2F_HIP(hipMemcpyAsync(v, r->net[net].trace, sizeof(double) * n, hipMemcpyDeviceToHost, r->stream));
    N2F_HIP(hipStreamSynchronize(r->stream));
    return N2F_OK;
}

n2f_status n2f_get_lohi(n2f_run* r, float* lo, float* hi) {
    if (!r) return fail(N2F_EINVAL, "run is NULL");
    if (lo) *lo = r->lo;
    if (hi) *hi = r->hi;
    return N2F_OK;
}

n2f_status n2f_get_image(n2f_run* r, int which, float* d_out) {
    if (!r || !d_out) return fail(N2F_EINVAL, "run or output is NULL");
    if (r->constant) return fail(N2F_ESTATE, "constant image: nothing prepared");
    const Plan& pl = r->pl;
    if (which >= 0 && which < 4) {
        const int h = which < 2 ? pl.hu : pl.hl, w = which < 2 ? pl.wu : pl.wl;
        N2F_HIP(launch_extract(r->ds[which], h, w, pl.C, d_out, r->stream));
    } else if (which == 4) {
        N2F_HIP(launch_extract(r->xs, pl.H, pl.W, pl.C, d_out, r->stream));
    } else if (which >= 5 && which < 5 + pl.C) {
        N2F_HIP(hipMemcpyAsync(d_out, r->net[which - 5].y, sizeof(float) * pl.H * pl.W, hipMemcpyDeviceToDevice,
                               r->stream));
    } else if (which >= 8 && which < 12) {
        if (pl.exact && !r->clean_set) return fail(N2F_ESTATE, "exact-target run: targets not built yet");
        const int p = which - 8;
        const int h = p < 2 ? pl.hu : pl.hl, w = p < 2 ? pl.wu : pl.wl;
        N2F_HIP(launch_extract(r->tg[p], h, w, pl.C, d_out, r->stream));
    } else {
        return fail(N2F_EINVAL, "unknown image index");
    }
    return N2F_OK;
}

n2f_status n2f_profile_begin(int every) {
    if (every < 1) return fail(N2F_EINVAL, "every must be >= 1");
    g_prof.recs.clear();
    g_prof.used = 0;
    g_prof.every = every;
    g_prof.epochs = 0;
    g_prof.on = true;
    return N2F_OK;
}

n2f_status n2f_profile_read(int cls, double* total_ms, long long* launches, long long* pixels) {
    if (!(cls >= N2F_K_CONV_FWD && cls <= N2F_K_ADAM) && !(cls >= N2F_K_GROUP && cls < N2F_K_GROUP + KK_COUNT))
        return fail(N2F_EINVAL, "unknown kernel class");
    double ms = 0.0;
    long long n = 0, px = 0;
    for (const ProfRec& rec : g_prof.recs) {
        if (rec.cls != cls) continue;
        N2F_HIP(hipEventSynchronize(rec.b));
        float t = 0.f;
        N2F_HIP(hipEventElapsedTime(&t, rec.a, rec.b));
        ms += t;
        n += rec.launches;
        px += rec.npix;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (pixels) *pixels = px;
    return N2F_OK;
}

n2f_status n2f_profile_end(void) {
    g_prof.on = false;
    return N2F_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch recording and grouped epochs
// ---------------------------------------------------------------------------
namespace n2f {

Recorder*& launch_recorder() {
    thread_local Recorder* r = nullptr;
    return r;
}

hipError_t record_launch(int kind, const void* args, size_t bytes, int grid, long long npix, int cost) {
    Recorder* r = launch_recorder();
    if (!r || bytes > (size_t)kArgStride || kind < 0 || kind >= KK_COUNT || grid < 1) return hipErrorInvalidValue;
    r->recs.emplace_back();
    LaunchRec& rec = r->recs.back();
    rec.kind = kind;
    rec.grid = grid;
    rec.npix = npix;
    rec.cost = std::max(1, cost);
    std::memset(rec.args, 0, sizeof(rec.args));
    std::memcpy(rec.args, args, bytes);
    return hipSuccess;
}

n2f_status record_epoch(n2f_run* r, int net, std::vector<LaunchRec>* out) {
    n2f_status s = check_run(r, net);
    if (s != N2F_OK) return s;
    if (!r->pl.bf) return fail(N2F_EINVAL, "grouped launches need BF16 runs");
    if (r->pl.gen) return fail(N2F_EINVAL, "grouped launches need the 64-wide network");
    s = check_targets(r);
    if (s != N2F_OK) return s;
    Recorder rec;
    launch_recorder() = &rec;
    const bool cap = g_prof.capturing;
    g_prof.capturing = true;   // no event brackets while recording
    s = enqueue_epoch(r, net);
    g_prof.capturing = cap;
    launch_recorder() = nullptr;
    if (s != N2F_OK) return s;
    *out = std::move(rec.recs);
    return N2F_OK;
}

hipStream_t run_stream(n2f_run* r) { return r->stream; }

bool profiling_on() { return g_prof.on; }

bool Group::next_epoch_timed() { return g_prof.on && (g_prof.epochs % g_prof.every) == 0; }

namespace {
// Blocks per grouped launch: the 3x3 kernels hold most of a CU's shared
// memory (one block per CU); the others are short memory-bound blocks.
int g_group_grid[KK_COUNT] = {256, 256, 256, 256, 256, 256, 1024, 1024, 1024, 512, 512, 512, 1024, 256, 1024};
}  // namespace

int group_grid(int kind) { return (kind >= 0 && kind < KK_COUNT) ? g_group_grid[kind] : 1; }
void set_group_grid(int kind, int grid) {
    if (kind >= 0 && kind < KK_COUNT && grid >= 1 && grid <= kMaxGroupGrid) g_group_grid[kind] = grid;
}

namespace {
// Layout of one launch position of a group's tables: the prefix (cap + 2
// ints), the block starts (kMaxGroupGrid + 1 ints), then cap argument blocks.
size_t head_bytes(int cap) { return align_up(sizeof(int) * (size_t)(cap + 2 + kMaxGroupGrid + 1)); }
}  // namespace

size_t Group::table_bytes(int cap) { return (size_t)kMaxPos * (head_bytes(cap) + (size_t)cap * kArgStride); }

size_t Group::pos_bytes() const { return head_bytes(cap_) + (size_t)cap_ * kArgStride; }

Group::~Group() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
}

n2f_status Group::add(n2f_run* r, int net, int tag) {
    if ((int)slots_.size() >= cap_) return fail(N2F_ENOMEM, "group is full (" + std::to_string(cap_) + " runs)");
    if (run_stream(r) != stream_) return fail(N2F_EINVAL, "a grouped run must be created on the group's stream");
    Slot sl{tag, r, net, {}};
    n2f_status s = record_epoch(r, net, &sl.recs);
    if (s != N2F_OK) return s;
    if (sl.recs.size() > (size_t)kMaxPos) return fail(N2F_EINVAL, "epoch has too many launches for a group");
    std::vector<int> kinds;
    for (const LaunchRec& rec : sl.recs) kinds.push_back(rec.kind);
    if (kinds_.empty()) {
        kinds_ = kinds;
    } else if (kinds != kinds_) {
        return fail(N2F_EINVAL, "the runs of a group must have the same launch sequence (channel count)");
    }
    slots_.push_back(std::move(sl));
    dirty_ = true;
    return N2F_OK;
}

n2f_status Group::set_net(int tag, int net) {
    for (Slot& sl : slots_) {
        if (sl.tag != tag) continue;
        std::vector<LaunchRec> recs;
        n2f_status s = record_epoch(sl.run, net, &recs);
        if (s != N2F_OK) return s;
        if (recs.size() != kinds_.size()) return fail(N2F_EINVAL, "launch sequence changed");
        sl.net = net;
        sl.recs = std::move(recs);
        dirty_ = true;
        return N2F_OK;
    }
    return fail(N2F_EINVAL, "no run with that tag in the group");
}

void Group::remove(int tag) {
    for (size_t i = 0; i < slots_.size(); ++i) {
        if (slots_[i].tag != tag) continue;
        slots_.erase(slots_.begin() + i);
        dirty_ = true;
        return;
    }
}

// Lay the runs' records out as per-launch tables and copy them to the device
// (on the stream, after the epochs already queued).  The host copy is only
// rewritten once the previous upload has completed.
n2f_status Group::upload() {
    N2F_HIP(hipStreamSynchronize(stream_));
    const int n = (int)slots_.size();
    const size_t pb = pos_bytes(), hb = head_bytes(cap_);
    const size_t npos = kinds_.size();
    host_.assign(npos * pb, 0);
    npix_.assign(npos, 0);
    for (size_t j = 0; j < npos; ++j) {
        unsigned char* base = host_.data() + j * pb;
        int* pf = reinterpret_cast<int*>(base);
        int* st = pf + cap_ + 2;
        pf[0] = n;
        pf[1] = 0;
        long long cost = 0;
        for (int i = 0; i < n; ++i) {
            const LaunchRec& rec = slots_[i].recs[j];
            pf[2 + i] = pf[1 + i] + rec.grid;
            std::memcpy(base + hb + (size_t)i * kArgStride, rec.args, kArgStride);
            npix_[j] += rec.npix;
            cost += (long long)rec.grid * rec.cost;
        }
        // block b starts at the first virtual block whose cost before it is
        // at least cost * b / G
        const int G = group_grid(kinds_[j]);
        long long before = 0;
        int gv = 0, b = 0;
        for (int i = 0; i < n; ++i) {
            const LaunchRec& rec = slots_[i].recs[j];
            for (int v = 0; v < rec.grid; ++v, ++gv) {
                while (b < G && before >= (cost * b + G - 1) / G) st[b++] = gv;
                before += rec.cost;
            }
        }
        while (b <= G) st[b++] = gv;
    }
    if (!host_.empty()) N2F_HIP(hipMemcpyAsync(d_tab_, host_.data(), host_.size(), hipMemcpyHostToDevice, stream_));
    dirty_ = false;
    return N2F_OK;
}

n2f_status Group::enqueue_all(hipStream_t s, bool with_timing) {
    const size_t pb = pos_bytes(), hb = head_bytes(cap_);
    for (size_t j = 0; j < kinds_.size(); ++j) {
        const int kind = kinds_[j];
        char* base = d_tab_ + j * pb;
        const GroupView v{reinterpret_cast<const unsigned char*>(base + hb), reinterpret_cast<const int*>(base),
                          reinterpret_cast<const int*>(base) + cap_ + 2};
        const int grid = group_grid(kind);
        if (with_timing) {
            N2F_HIP(timed(N2F_K_GROUP + kind, 1, npix_[j], s, [&] { return launch_group(kind, v, grid, s); }));
        } else {
            N2F_HIP(launch_group(kind, v, grid, s));
        }
    }
    return N2F_OK;
}

n2f_status Group::launch(int epochs) {
    if (slots_.empty() || epochs < 1) return N2F_OK;
    bool stale = exec_ == nullptr;
    for (int k = 0; k < KK_COUNT; ++k) stale = stale || exec_grid_[k] != group_grid(k);
    if (dirty_ || stale) {   // the block starts depend on the grids too
        n2f_status s = upload();
        if (s != N2F_OK) return s;
    }
    if (stale) {
        // record one epoch of grouped launches on a private stream; the
        // tables it points at are rewritten in place, never moved
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
        if (!cap_stream_) N2F_HIP(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        const bool capf = g_prof.capturing;
        g_prof.capturing = true;
        hipError_t e = hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeRelaxed);
        n2f_status s = N2F_OK;
        if (e == hipSuccess) s = enqueue_all(cap_stream_, false);
        hipGraph_t g = nullptr;
        hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(cap_stream_, &g) : e;
        g_prof.capturing = capf;
        if (e != hipSuccess || e2 != hipSuccess || s != N2F_OK) {
            if (g) (void)hipGraphDestroy(g);
            if (s != N2F_OK) return s;
            return fail(N2F_EDEVICE, std::string("group graph capture failed: ") +
                                         hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            exec_ = nullptr;
            return fail(N2F_EDEVICE, std::string("group graph instantiate failed: ") + hipGetErrorString(e));
        }
        graph_ = g;
        for (int k = 0; k < KK_COUNT; ++k) exec_grid_[k] = group_grid(k);
    }
    for (int e = 0; e < epochs; ++e) {
        const bool direct = g_prof.on && (g_prof.epochs++ % g_prof.every) == 0;
        if (direct) {
            n2f_status s = enqueue_all(stream_, true);
            if (s != N2F_OK) return s;
        } else {
            N2F_HIP(hipGraphLaunch(exec_, stream_));
        }
    }
    return N2F_OK;
}

}  // namespace n2f

extern "C" {

n2f_status n2f_group_grid_get(int kind, int* grid) {
    if (kind < 0 || kind >= KK_COUNT || !grid) return fail(N2F_EINVAL, "grouped kind out of range or grid is NULL");
    *grid = group_grid(kind);
    return N2F_OK;
}

n2f_status n2f_group_grid_set(int kind, int grid) {
    if (kind < 0 || kind >= KK_COUNT) return fail(N2F_EINVAL, "grouped kind out of range");
    if (grid < 1 || grid > kMaxGroupGrid) return fail(N2F_EINVAL, "grid must be in 1.." + std::to_string(kMaxGroupGrid));
    set_group_grid(kind, grid);
    return N2F_OK;
}

}  // extern "C"
