// Scheduling of many independent Noise2Fast runs on one GPU: a fixed batch
// of images of uneven sizes, and a continuous-batching server that admits
// requests by device-memory budget and lets runs join and leave at epoch
// boundaries.  Built on the public run API of include/n2f.h: every run
// replays its own recorded epoch graph on one of a few HIP streams, so the
// epochs of different images overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "n2f.h"
#include "n2f_internal.h"

namespace {

n2f_status sfail(n2f_status code, const std::string& msg) {
    n2f::set_last_error(msg);
    return code;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Epochs queued per run between two polls of its stopping rule.
constexpr int kPollEpochs = 4;

n2f_status make_streams(std::vector<hipStream_t>& v, int n) {
    for (int i = 0; i < n; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
            return sfail(N2F_EDEVICE, "stream creation failed");
        v.push_back(s);
    }
    return N2F_OK;
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
   public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t largest() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t size() const { return size_; }

   private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length
};

}  // namespace

// ---------------------------------------------------------------------------
// Batch
// ---------------------------------------------------------------------------
struct n2f_batch {
    n2f_config cfg;
    int n = 0;
    std::vector<n2f_run*> runs;
    std::vector<int> C, net, finished, epochs, stream_of, removed;
    std::vector<long long> work;   // pixels x channels of each image
    std::vector<int> status;   // N2F_ENUMERIC once a network of the image failed
    std::vector<hipStream_t> streams;
    bool own_streams = true;   // false: the batch runs on the caller's stream alone
    hipStream_t caller = nullptr;
    // grouped mode: one group per (channel count, batch stream), tables after
    // the images; group of image i: groups[3 * stream_of[i] + C[i] - 1]
    bool grouped = false;
    int group_cap = 0;
    char* tables = nullptr;
    std::vector<std::unique_ptr<n2f::Group>> groups;
    n2f::Group* group_of(int i) { return groups[3 * stream_of[i] + C[i] - 1].get(); }
    ~n2f_batch() {
        if (grouped)
            for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
        for (auto& g : groups) g.reset();
        for (n2f_run* r : runs)
            if (r) n2f_run_destroy(r);
        if (own_streams)
            for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }
};

namespace {

// Make stream `s` wait for the work queued on `caller` so far.
n2f_status order_after(hipStream_t s, hipStream_t caller) {
    if (s == caller) return N2F_OK;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return sfail(N2F_EDEVICE, "event creation failed");
    hipError_t e = hipEventRecord(ev, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    (void)hipEventDestroy(ev);   // released once the wait has been satisfied
    return e == hipSuccess ? N2F_OK : sfail(N2F_EDEVICE, "stream ordering failed");
}

constexpr int kGroupExtra = 64;   // images a grouped batch can take beyond its initial n
constexpr int kMaxGroupStreams = 4;   // streams of a grouped batch (n_streams = -1 .. -4)

size_t batch_table_bytes(int n) {
    return (size_t)3 * kMaxGroupStreams * align_up(n2f::Group::table_bytes(n + kGroupExtra));
}

// Grouped mode: image i (created, not finished) joins the group of its
// channel count on its stream, created on first use.
n2f_status group_join(n2f_batch* b, int i) {
    const int gi = 3 * b->stream_of[i] + b->C[i] - 1;
    if (!b->groups[gi]) {
        b->groups[gi].reset(new (std::nothrow) n2f::Group(
            b->group_cap, b->tables + gi * align_up(n2f::Group::table_bytes(b->group_cap)),
            b->streams[b->stream_of[i]]));
        if (!b->groups[gi]) return sfail(N2F_ENOMEM, "host allocation failed");
    }
    return b->groups[gi]->add(b->runs[i], b->net[i], i);
}

// Create the run of a new batch image on the least loaded stream (by work)
// and append it; *index receives its index.
n2f_status batch_append(n2f_batch* b, const float* d_in, int H, int W, int C, void* ws, size_t wb, int* index) {
    const int ns = (int)b->streams.size();
    std::vector<long long> load(ns, 0);
    for (int i = 0; i < b->n; ++i)
        if (!b->removed[i] && !b->finished[i]) load[b->stream_of[i]] += b->work[i];
    const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    n2f_status s = order_after(b->streams[si], b->caller);
    if (s != N2F_OK) return s;
    n2f_run* r = nullptr;
    s = n2f_run_create(&r, d_in, H, W, C, &b->cfg, ws, wb, b->streams[si]);
    if (s < 0) return s;
    b->runs.push_back(r);
    b->C.push_back(C);
    b->net.push_back(0);
    b->finished.push_back(s == N2F_WCONSTANT ? 1 : 0);
    b->epochs.push_back(0);
    b->stream_of.push_back(si);
    b->removed.push_back(0);
    b->work.push_back((long long)H * W * C);
    b->status.push_back(N2F_OK);
    const int i = b->n++;
    if (index) *index = i;
    if (b->grouped && !b->finished[i]) {
        s = group_join(b, i);
        if (s != N2F_OK) {
            n2f_run_destroy(b->runs[i]);
            b->runs[i] = nullptr;
            b->removed[i] = 1;
            b->finished[i] = 1;
            return s;
        }
    }
    return N2F_OK;
}

}  // namespace

namespace {

// Grouped mode: the groups of each stream replay whole epochs there, then
// the host reads the stopping rule of that stream's images; a finished
// network leaves its group (or moves on to the image's next network), and
// the group's tables are rewritten before its next epochs.  Streams are
// served in turn, each refed as soon as its own epochs are read, so groups
// on different streams drift to different points of their epochs and their
// launches of different kinds overlap.
n2f_status batch_run_grouped(n2f_batch* b, int max_now) {
    const int ns = (int)b->streams.size();
    std::vector<int> ran(ns, 0);
    // a timed epoch (kernel timing on) has the GPU to itself: its stream
    // first waits for the work queued on the others, and they wait for it,
    // so the timed launches are not slowed by concurrent ones
    auto fence = [&](int s, bool before) -> n2f_status {
        for (int t = 0; t < ns; ++t) {
            if (t == s) continue;
            n2f_status st = before ? order_after(b->streams[s], b->streams[t]) : order_after(b->streams[t], b->streams[s]);
            if (st != N2F_OK) return st;
        }
        return N2F_OK;
    };
    auto feed = [&](int s, bool* fed) -> n2f_status {
        *fed = false;
        if (ran[s] >= max_now) return N2F_OK;
        const int k = std::min(n2f::profiling_on() ? 1 : kPollEpochs, max_now - ran[s]);
        for (int c = 0; c < 3; ++c) {
            n2f::Group* g = b->groups[3 * s + c].get();
            if (!g || g->size() == 0) continue;
            const bool excl = ns > 1 && n2f::Group::next_epoch_timed();
            n2f_status st = excl ? fence(s, true) : N2F_OK;
            if (st != N2F_OK) return st;
            st = g->launch(k);
            if (st < 0) return st;
            if (excl) {
                st = fence(s, false);
                if (st != N2F_OK) return st;
            }
            *fed = true;
        }
        if (*fed) ran[s] += k;
        return N2F_OK;
    };
    auto drain = [&](int s) -> n2f_status {
        for (int i = 0; i < b->n; ++i) {
            if (b->finished[i] || b->stream_of[i] != s) continue;
            n2f::Group* g = b->group_of(i);
            int done = 0, ep = 0;
            n2f_status st = n2f_run_poll(b->runs[i], b->net[i], &done, &ep);
            if (st == N2F_ENUMERIC) {
                b->epochs[i] += ep;
                b->status[i] = st;
                b->finished[i] = 1;
                g->remove(i);
                continue;
            }
            if (st < 0) return st;
            if (!done) continue;
            b->epochs[i] += ep;
            if (++b->net[i] >= b->C[i]) {
                b->finished[i] = 1;
                g->remove(i);
            } else {
                st = g->set_net(i, b->net[i]);
                if (st < 0) return st;
            }
        }
        return N2F_OK;
    };
    std::vector<char> pending(ns, 0);
    bool any = false;
    for (int s = 0; s < ns; ++s) {
        bool fed = false;
        n2f_status st = feed(s, &fed);
        if (st < 0) return st;
        pending[s] = fed;
        any = any || fed;
    }
    while (any) {
        any = false;
        for (int s = 0; s < ns; ++s) {
            if (!pending[s]) continue;
            n2f_status st = drain(s);
            if (st < 0) return st;
            bool fed = false;
            st = feed(s, &fed);
            if (st < 0) return st;
            pending[s] = fed;
            any = any || fed;
        }
    }
    return N2F_OK;
}

}  // namespace

extern "C" {

n2f_status n2f_batch_workspace_bytes(int n, const int* H, const int* W, const int* C, const n2f_config* cfg,
                                     size_t* bytes) {
    if (n < 1 || !H || !W || !C || !bytes) return sfail(N2F_EINVAL, "bad batch arguments");
    size_t tot = 0;
    for (int i = 0; i < n; ++i) {
        size_t b = 0;
        n2f_status s = n2f_workspace_bytes(H[i], W[i], C[i], cfg, &b);
        if (s != N2F_OK) return s;
        tot += align_up(b);
    }
    *bytes = tot + batch_table_bytes(n);
    return N2F_OK;
}

n2f_status n2f_batch_create(n2f_batch** out, int n, const float* const* d_in, const int* H, const int* W,
                            const int* C, const n2f_config* cfg, void* d_ws, size_t ws_bytes, int n_streams,
                            hipStream_t stream) {
    if (!out || !d_in || !d_ws || !cfg || n < 1 || n_streams < -kMaxGroupStreams)
        return sfail(N2F_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (cfg->exact_targets) return sfail(N2F_EINVAL, "exact targets need a clean image per run: not in a batch");
    if (n_streams <= N2F_BATCH_GROUPED && cfg->precision != N2F_BF16)
        return sfail(N2F_EINVAL, "grouped batches need BF16 (the FP32 path has no grouped kernels)");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return sfail(N2F_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    n2f_status s = n2f_batch_workspace_bytes(n, H, W, C, cfg, &need);
    if (s != N2F_OK) return s;
    if (ws_bytes < need) return sfail(N2F_ENOMEM, "batch workspace too small");
    n2f_batch* b = new (std::nothrow) n2f_batch();
    if (!b) return sfail(N2F_ENOMEM, "host allocation failed");
    b->cfg = *cfg;
    b->caller = stream;
    if (n_streams <= N2F_BATCH_GROUPED) {
        b->grouped = true;
        b->group_cap = n + kGroupExtra;
        b->tables = static_cast<char*>(d_ws) + (need - batch_table_bytes(n));
        b->groups.resize(3 * kMaxGroupStreams);
        if (n_streams == N2F_BATCH_GROUPED) {   // the caller's stream
            b->own_streams = false;
            b->streams.push_back(stream);
        } else {
            s = make_streams(b->streams, -n_streams);
            if (s != N2F_OK) {
                delete b;
                return s;
            }
        }
    } else if (n_streams == 0) {
        b->own_streams = false;
        b->streams.push_back(stream);
    } else {
        s = make_streams(b->streams, std::min(n, n_streams));
        if (s != N2F_OK) {
            delete b;
            return s;
        }
    }
    // images largest first onto the least loaded stream (pixels x channels:
    // each channel is one network trained in turn); indices keep the
    // caller's order
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    auto work = [&](int i) { return (long long)H[i] * W[i] * C[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
    std::vector<size_t> off(n);
    size_t o = 0;
    for (int i = 0; i < n; ++i) {
        size_t wb = 0;
        n2f_workspace_bytes(H[i], W[i], C[i], cfg, &wb);
        off[i] = o;
        o += align_up(wb);
    }
    // create in the caller's order, with the stream chosen by the sorted pass
    const int ns = (int)b->streams.size();
    std::vector<int> stream_of(n);
    std::vector<long long> load(ns, 0);
    for (int i : order) {
        const int si = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        stream_of[i] = si;
        load[si] += work(i);
    }
    for (int si = 0; si < ns; ++si) {
        s = order_after(b->streams[si], stream);
        if (s != N2F_OK) {
            delete b;
            return s;
        }
    }
    char* ws = static_cast<char*>(d_ws);
    for (int i = 0; i < n; ++i) {
        size_t wb = 0;
        n2f_workspace_bytes(H[i], W[i], C[i], cfg, &wb);
        const int si = stream_of[i];
        n2f_run* r = nullptr;
        s = n2f_run_create(&r, d_in[i], H[i], W[i], C[i], cfg, ws + off[i], wb, b->streams[si]);
        if (s < 0) {
            delete b;
            return s;
        }
        b->runs.push_back(r);
        b->C.push_back(C[i]);
        b->net.push_back(0);
        b->finished.push_back(s == N2F_WCONSTANT ? 1 : 0);
        b->epochs.push_back(0);
        b->stream_of.push_back(si);
        b->removed.push_back(0);
        b->work.push_back(work(i));
        b->status.push_back(N2F_OK);
        b->n++;
        if (b->grouped && !b->finished[i]) {
            s = group_join(b, i);
            if (s != N2F_OK) {
                delete b;
                return s;
            }
        }
    }
    *out = b;
    return N2F_OK;
}

n2f_status n2f_batch_add(n2f_batch* b, const float* d_in, int H, int W, int C, void* d_ws, size_t ws_bytes,
                         int* index) {
    if (!b || !d_in || !d_ws) return sfail(N2F_EINVAL, "bad batch arguments");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return sfail(N2F_EINVAL, "workspace must be 256-byte aligned");
    size_t wb = 0;
    n2f_status s = n2f_workspace_bytes(H, W, C, &b->cfg, &wb);
    if (s != N2F_OK) return s;
    if (ws_bytes < wb) return sfail(N2F_ENOMEM, "workspace too small: need " + std::to_string(wb) + " bytes");
    return batch_append(b, d_in, H, W, C, d_ws, wb, index);
}

n2f_status n2f_batch_remove(n2f_batch* b, int i) {
    if (!b || i < 0 || i >= b->n) return sfail(N2F_EINVAL, "bad batch arguments");
    if (b->removed[i]) return sfail(N2F_ESTATE, "image " + std::to_string(i) + " already removed");
    if (hipStreamSynchronize(b->streams[b->stream_of[i]]) != hipSuccess) return sfail(N2F_EDEVICE, "sync failed");
    if (b->grouped && b->group_of(i)) b->group_of(i)->remove(i);
    n2f_run_destroy(b->runs[i]);
    b->runs[i] = nullptr;
    b->removed[i] = 1;
    b->finished[i] = 1;
    return N2F_OK;
}

n2f_status n2f_batch_run(n2f_batch* b, int max_now, int* n_active) {
    if (!b || max_now < 1) return sfail(N2F_EINVAL, "bad batch arguments");
    if (b->grouped) {
        n2f_status st = batch_run_grouped(b, max_now);
        if (st < 0) return st;
        if (n_active) {
            int a = 0;
            for (int i = 0; i < b->n; ++i) a += !b->finished[i];
            *n_active = a;
        }
        return N2F_OK;
    }
    std::vector<int> ran(b->n, 0);
    const int ns = (int)b->streams.size();
    std::vector<std::vector<int>> on(ns);   // images of each stream
    for (int i = 0; i < b->n; ++i) on[b->stream_of[i]].push_back(i);
    // queue a few epochs for every image of stream s still training; the
    // number of images queued, or an error
    auto feed = [&](int s, int* queued) -> n2f_status {
        *queued = 0;
        for (int i : on[s]) {
            if (b->finished[i] || ran[i] >= max_now) continue;
            const int k = std::min(kPollEpochs, max_now - ran[i]);
            n2f_status st = n2f_run_launch_epochs(b->runs[i], b->net[i], k);
            if (st < 0) return st;
            ran[i] += k;
            ++*queued;
        }
        return N2F_OK;
    };
    // read the stopping rule of every image of stream s (waits for the
    // stream's queued epochs); an image whose score turned non-finite fails
    // alone, the others go on
    auto drain = [&](int s) -> n2f_status {
        for (int i : on[s]) {
            if (b->finished[i]) continue;
            int done = 0, ep = 0;
            n2f_status st = n2f_run_poll(b->runs[i], b->net[i], &done, &ep);
            if (st == N2F_ENUMERIC) {
                b->epochs[i] += ep;
                b->status[i] = st;
                b->finished[i] = 1;
                continue;
            }
            if (st < 0) return st;
            if (done) {
                b->epochs[i] += ep;
                if (++b->net[i] >= b->C[i]) b->finished[i] = 1;
            }
        }
        return N2F_OK;
    };
    // every stream gets work, then the streams are served in turn: while
    // the host waits for one and queues its next epochs, the others run, so
    // no stream waits for the slowest one as it would with a common round
    std::vector<char> busy(ns, 0);
    for (int s = 0; s < ns; ++s) {
        int q = 0;
        n2f_status st = feed(s, &q);
        if (st < 0) return st;
        busy[s] = q > 0;
    }
    for (bool any = true; any;) {
        any = false;
        for (int s = 0; s < ns; ++s) {
            if (!busy[s]) continue;
            any = true;
            n2f_status st = drain(s);
            if (st < 0) return st;
            int q = 0;
            st = feed(s, &q);
            if (st < 0) return st;
            busy[s] = q > 0;
        }
    }
    if (n_active) {
        int a = 0;
        for (int i = 0; i < b->n; ++i) a += !b->finished[i];
        *n_active = a;
    }
    return N2F_OK;
}

n2f_status n2f_batch_result(n2f_batch* b, int i, float* d_out) {
    if (!b || i < 0 || i >= b->n || !d_out) return sfail(N2F_EINVAL, "bad batch arguments");
    if (b->removed[i]) return sfail(N2F_ESTATE, "image " + std::to_string(i) + " was removed");
    if (b->status[i] < 0) return sfail(b->status[i], "image " + std::to_string(i) + ": validation score not finite");
    n2f_status s = n2f_result(b->runs[i], d_out);
    if (s < 0) return s;
    if (hipStreamSynchronize(b->streams[b->stream_of[i]]) != hipSuccess) return sfail(N2F_EDEVICE, "sync failed");
    return s;
}

n2f_status n2f_batch_run_of(n2f_batch* b, int i, n2f_run** run) {
    if (!b || i < 0 || i >= b->n || !run) return sfail(N2F_EINVAL, "bad batch arguments");
    if (b->removed[i]) return sfail(N2F_ESTATE, "image " + std::to_string(i) + " was removed");
    *run = b->runs[i];
    return N2F_OK;
}

n2f_status n2f_batch_progress(n2f_batch* b, int i, int* epochs, int* finished) {
    if (!b || i < 0 || i >= b->n) return sfail(N2F_EINVAL, "bad batch arguments");
    int ep = b->epochs[i];
    if (!b->finished[i] && !b->removed[i] && b->net[i] < b->C[i]) {
        int cur = 0;
        if (n2f_get_progress(b->runs[i], b->net[i], &cur, nullptr, nullptr, nullptr) == N2F_OK) ep += cur;
    }
    if (epochs) *epochs = ep;
    if (finished) *finished = b->finished[i];
    return N2F_OK;
}

n2f_status n2f_batch_destroy(n2f_batch* b) {
    if (!b) return sfail(N2F_EINVAL, "batch is NULL");
    delete b;
    return N2F_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------
struct n2f_server {
    struct Req {
        long long id;
        const float* in;
        float* out;
        int H, W, C, sim_epochs;
        size_t bytes;
        hipEvent_t ready;   // recorded on the submitter's stream: the input is complete
    };
    struct Active {
        Req q;
        n2f_run* run;
        size_t off;
        int net, stream, epochs;
        int tag;   // grouped mode: the run's tag in its group
    };
    n2f_config cfg;
    char* arena_base = nullptr;   // where request workspaces start (after the tables in grouped mode)
    Arena arena;
    bool simulate = false;
    bool grouped = false;
    int max_active = 1;
    int next_tag = 0;
    std::unique_ptr<n2f::Group> groups[3];
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;
    std::deque<Req> queue;
    std::vector<Active> active;
    std::deque<std::pair<long long, int>> finished;
    explicit n2f_server(size_t bytes) : arena(bytes) {}
    ~n2f_server() {
        for (hipStream_t s : streams) (void)hipStreamSynchronize(s);   // queued epochs end first
        for (auto& g : groups) g.reset();
        for (Active& a : active)
            if (a.run) n2f_run_destroy(a.run);
        for (Req& q : queue)
            if (q.ready) (void)hipEventDestroy(q.ready);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }
};

namespace {

// Finish active request idx with `status`: destroy its run, free its arena
// range, report its id.
void retire(n2f_server* v, size_t idx, int status) {
    n2f_server::Active& a = v->active[idx];
    if (v->grouped && a.run && v->groups[a.q.C - 1]) v->groups[a.q.C - 1]->remove(a.tag);
    if (a.run) n2f_run_destroy(a.run);
    v->arena.release(a.off, a.q.bytes);
    if (!v->simulate) v->stream_load[a.stream]--;
    v->finished.emplace_back(a.q.id, status);
    v->active.erase(v->active.begin() + idx);
}

}  // namespace

extern "C" {

n2f_status n2f_server_table_bytes(int max_active, size_t* bytes) {
    if (max_active < 1 || !bytes) return sfail(N2F_EINVAL, "bad server arguments");
    *bytes = 3 * align_up(n2f::Group::table_bytes(max_active));
    return N2F_OK;
}

n2f_status n2f_server_create(n2f_server** out, const n2f_config* cfg, void* d_arena, size_t arena_bytes,
                             int n_streams, int max_active, int flags) {
    if (!out || !cfg || max_active < 1) return sfail(N2F_EINVAL, "bad server arguments");
    const bool grouped = (flags & N2F_SERVER_GROUPED) != 0;
    if (!grouped && n_streams < 1) return sfail(N2F_EINVAL, "n_streams must be >= 1");
    if (cfg->exact_targets) return sfail(N2F_EINVAL, "exact targets need a clean image per run: not served");
    if (grouped && cfg->precision != N2F_BF16)
        return sfail(N2F_EINVAL, "grouped serving needs BF16 (the FP32 path has no grouped kernels)");
    const bool sim = (flags & N2F_SERVER_SIMULATE) != 0;
    const size_t tables = grouped ? 3 * align_up(n2f::Group::table_bytes(max_active)) : 0;
    if (tables >= arena_bytes) return sfail(N2F_ENOMEM, "arena smaller than the grouped launch tables");
    if (!sim && !d_arena) return sfail(N2F_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(d_arena) % kAlign) return sfail(N2F_EINVAL, "arena must be 256-byte aligned");
    size_t probe = 0;
    n2f_status s = n2f_workspace_bytes(2, 2, 1, cfg, &probe);   // validates the config
    if (s != N2F_OK) return s;
    n2f_server* v = new (std::nothrow) n2f_server(arena_bytes - tables);
    if (!v) return sfail(N2F_ENOMEM, "host allocation failed");
    v->cfg = *cfg;
    v->arena_base = static_cast<char*>(d_arena) + tables;
    v->simulate = sim;
    v->grouped = grouped && !sim;
    v->max_active = max_active;
    if (!sim) {
        s = make_streams(v->streams, grouped ? 1 : n_streams);
        if (s != N2F_OK) {
            delete v;
            return s;
        }
        v->stream_load.assign(v->streams.size(), 0);
        if (v->grouped) {
            for (int c = 0; c < 3; ++c) {
                v->groups[c].reset(new (std::nothrow) n2f::Group(
                    max_active, static_cast<char*>(d_arena) + c * align_up(n2f::Group::table_bytes(max_active)),
                    v->streams[0]));
                if (!v->groups[c]) {
                    delete v;
                    return sfail(N2F_ENOMEM, "host allocation failed");
                }
            }
        }
    }
    *out = v;
    return N2F_OK;
}

n2f_status n2f_server_submit(n2f_server* v, long long id, const float* d_in, float* d_out, int H, int W, int C,
                             int sim_epochs, hipStream_t stream) {
    if (!v) return sfail(N2F_EINVAL, "server is NULL");
    if (!v->simulate && (!d_in || !d_out)) return sfail(N2F_EINVAL, "input or output is NULL");
    size_t bytes = 0;
    n2f_status s = n2f_workspace_bytes(H, W, C, &v->cfg, &bytes);
    if (s != N2F_OK) return s;
    if (align_up(bytes) > v->arena.size()) return sfail(N2F_ENOMEM, "request can never fit in the arena");
    for (const n2f_server::Req& q : v->queue)
        if (q.id == id) return sfail(N2F_EINVAL, "id " + std::to_string(id) + " is already queued");
    for (const n2f_server::Active& a : v->active)
        if (a.q.id == id) return sfail(N2F_EINVAL, "id " + std::to_string(id) + " is already active");
    hipEvent_t ev = nullptr;
    if (!v->simulate) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return sfail(N2F_EDEVICE, "event creation failed");
        if (hipEventRecord(ev, stream) != hipSuccess) {
            (void)hipEventDestroy(ev);
            return sfail(N2F_EDEVICE, "event record failed");
        }
    }
    v->queue.push_back({id, d_in, d_out, H, W, C, std::max(1, sim_epochs), bytes, ev});
    return N2F_OK;
}

n2f_status n2f_server_cancel(n2f_server* v, long long id) {
    if (!v) return sfail(N2F_EINVAL, "server is NULL");
    for (auto it = v->queue.begin(); it != v->queue.end(); ++it) {
        if (it->id != id) continue;
        if (it->ready) (void)hipEventDestroy(it->ready);
        v->queue.erase(it);
        v->finished.emplace_back(id, N2F_ECANCELED);
        return N2F_OK;
    }
    for (size_t i = 0; i < v->active.size(); ++i) {
        if (v->active[i].q.id != id) continue;
        // the run's queued epochs finish before its arena range is reused
        if (!v->simulate && hipStreamSynchronize(v->streams[v->active[i].stream]) != hipSuccess)
            return sfail(N2F_EDEVICE, "sync failed");
        retire(v, i, N2F_ECANCELED);
        return N2F_OK;
    }
    return sfail(N2F_EINVAL, "no queued or active request with id " + std::to_string(id));
}

n2f_status n2f_server_step(n2f_server* v, int epochs, int* n_active, int* n_queued) {
    if (!v || epochs < 1) return sfail(N2F_EINVAL, "bad server arguments");
    // 1. admission, strictly in arrival order
    while (!v->queue.empty() && (int)v->active.size() < v->max_active) {
        n2f_server::Req q = v->queue.front();
        size_t off = 0;
        if (!v->arena.alloc(q.bytes, &off)) break;
        v->queue.pop_front();
        n2f_server::Active a{q, nullptr, off, 0, 0, 0};
        if (!v->simulate) {
            a.stream = (int)(std::min_element(v->stream_load.begin(), v->stream_load.end()) - v->stream_load.begin());
            v->stream_load[a.stream]++;
            hipError_t e = hipStreamWaitEvent(v->streams[a.stream], q.ready, 0);
            (void)hipEventDestroy(q.ready);
            if (e != hipSuccess) {
                v->active.push_back(a);
                retire(v, v->active.size() - 1, sfail(N2F_EDEVICE, "stream ordering failed"));
                continue;
            }
            n2f_status s = n2f_run_create(&a.run, q.in, q.H, q.W, q.C, &v->cfg, v->arena_base + off, q.bytes,
                                          v->streams[a.stream]);
            if (s < 0 || s == N2F_WCONSTANT) {
                if (s == N2F_WCONSTANT) s = n2f_result(a.run, q.out);
                (void)hipStreamSynchronize(v->streams[a.stream]);
                v->active.push_back(a);
                retire(v, v->active.size() - 1, s);
                continue;
            }
            if (v->grouped) {
                a.tag = v->next_tag++;
                s = v->groups[q.C - 1]->add(a.run, 0, a.tag);
                if (s != N2F_OK) {
                    n2f_run_destroy(a.run);
                    a.run = nullptr;
                    v->active.push_back(a);
                    retire(v, v->active.size() - 1, s);
                    continue;
                }
            }
        }
        v->active.push_back(a);
    }
    // 2. queue epochs for every active run (grouped: one launch sequence
    // per channel count covers them all)
    if (v->grouped) {
        for (auto& g : v->groups) {
            if (g->size() == 0) continue;
            n2f_status s = g->launch(epochs);
            if (s < 0) return s;
        }
    }
    for (n2f_server::Active& a : v->active) {
        if (v->simulate) {
            a.epochs += epochs;
            continue;
        }
        if (v->grouped) continue;
        n2f_status s = n2f_run_launch_epochs(a.run, a.net, epochs);
        if (s < 0) return s;
    }
    // 3. retire finished runs (result, arena range, id)
    for (size_t i = 0; i < v->active.size();) {
        n2f_server::Active& a = v->active[i];
        if (v->simulate) {
            if (a.epochs >= a.q.sim_epochs) {
                retire(v, i, N2F_OK);
                continue;
            }
            ++i;
            continue;
        }
        int done = 0;
        n2f_status s = n2f_run_poll(a.run, a.net, &done, nullptr);
        if (s < 0) {
            retire(v, i, s);
            continue;
        }
        if (done && ++a.net >= a.q.C) {
            s = n2f_result(a.run, a.q.out);
            if (hipStreamSynchronize(v->streams[a.stream]) != hipSuccess) s = sfail(N2F_EDEVICE, "sync failed");
            retire(v, i, s);
            continue;
        }
        if (done && v->grouped) {   // the request's next network joins the group
            s = v->groups[a.q.C - 1]->set_net(a.tag, a.net);
            if (s < 0) {
                retire(v, i, s);
                continue;
            }
        }
        ++i;
    }
    if (n_active) *n_active = (int)v->active.size();
    if (n_queued) *n_queued = (int)v->queue.size();
    return N2F_OK;
}

n2f_status n2f_server_poll(n2f_server* v, long long* ids, int* status, int max, int* n) {
    if (!v || !n || (max > 0 && !ids)) return sfail(N2F_EINVAL, "bad server arguments");
    int k = 0;
    while (k < max && !v->finished.empty()) {
        ids[k] = v->finished.front().first;
        if (status) status[k] = v->finished.front().second;
        v->finished.pop_front();
        ++k;
    }
    *n = k;
    return N2F_OK;
}

n2f_status n2f_server_memory(n2f_server* v, size_t* used, size_t* largest_free) {
    if (!v) return sfail(N2F_EINVAL, "server is NULL");
    if (used) *used = v->arena.used();
    if (largest_free) *largest_free = v->arena.largest();
    return N2F_OK;
}

n2f_status n2f_server_destroy(n2f_server* v) {
    if (!v) return sfail(N2F_EINVAL, "server is NULL");
    delete v;
    return N2F_OK;
}

}  // extern "C"
