// Host-side checks of libn2f's CPU-only paths, meant to be built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code (the
// device code is built as usual and never runs here): configuration checks,
// plans and workspace sizes over many shapes and configurations, the initial
// weights, the continuous-batching server's admission and arena bookkeeping
// in simulation mode over a long random trace, and the argument checks of the
// entry points.  Prints "host checks passed" and returns 0 on success.
#include <cmath>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "n2f.h"

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

static int config_checks() {
    n2f_config d;
    n2f_config_default(&d);
    size_t b = 0;
    CHECK(n2f_workspace_bytes(64, 64, 1, &d, &b) == N2F_OK && b > 0);
    n2f_config c = d;
    c.n_layers = 7;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.width = 40;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.widths[0] = 32;   // the other seven stay zero
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.lr = 0.f;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.beta2 = 1.0;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.pair_order[3] = 0;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.downsample = 5;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    c = d;
    c.exact_targets = -1;
    CHECK(n2f_workspace_bytes(64, 64, 1, &c, &b) == N2F_EINVAL);
    CHECK(n2f_workspace_bytes(64, 64, 1, nullptr, &b) == N2F_EINVAL);
    CHECK(n2f_workspace_bytes(64, 64, 1, &d, nullptr) == N2F_EINVAL);
    CHECK(n2f_workspace_bytes(1, 64, 1, &d, &b) == N2F_EINVAL);
    CHECK(n2f_workspace_bytes(64, 64, 4, &d, &b) == N2F_EINVAL);
    CHECK(n2f_workspace_bytes(1 << 15, 1 << 15, 1, &d, &b) == N2F_EINVAL);   // above 2^28 pixels
    CHECK(n2f_last_error()[0] != '\0');
    return 0;
}

static int plan_checks() {
    n2f_config d;
    n2f_config_default(&d);
    const int sides[] = {2, 3, 4, 5, 16, 17, 31, 64, 100, 255, 256, 511, 512, 1023, 2048, 4096};
    const int literal[8] = {32, 32, 64, 64, 128, 128, 256, 256};
    for (int lit = 0; lit < 2; ++lit)
    for (int prec = 0; prec < 2; ++prec)
        for (int ds = 0; ds < 2; ++ds)
            for (int ex = 0; ex < 2; ++ex)
                for (int C = 1; C <= 3; ++C)
                    for (int H : sides)
                        for (int W : sides) {
                            if (lit && (H > 1024 || W > 1024)) continue;
                            n2f_config c = d;
                            c.precision = prec;
                            c.downsample = ds;
                            c.exact_targets = ex;
                            if (lit)
                                for (int l = 0; l < 8; ++l) c.widths[l] = literal[l];
                            size_t b = 0, b2 = 0;
                            CHECK(n2f_workspace_bytes(H, W, C, &c, &b) == N2F_OK);
                            CHECK(b % 256 == 0);
                            // at least the stashed activations of the training image
                            const size_t P = ds ? (size_t)(H / 2) * (W / 2) : (size_t)(H & ~1) * (W & ~1) / 2;
                            CHECK(b >= P * (lit ? 992 : 64 * 8) * (prec ? 2 : 4));
                            if (ex) {
                                c.exact_targets = 0;
                                CHECK(n2f_workspace_bytes(H, W, C, &c, &b2) == N2F_OK && b2 < b);
                            }
                        }
    return 0;
}

static int param_checks() {
    n2f_config d;
    n2f_config_default(&d);
    for (int C = 1; C <= 3; ++C) {
        size_t n = 0;
        CHECK(n2f_param_count(C, &d, &n) == N2F_OK);
        CHECK(n == (size_t)(64 * C * 9 + 64) + 7 * (64 * 64 * 9 + 64) + 65);
        std::vector<float> a(C * n), b(C * n);
        CHECK(n2f_init_params(C, &d, 7, a.data()) == N2F_OK);
        CHECK(n2f_init_params(C, &d, 7, b.data()) == N2F_OK);
        CHECK(a == b);
        const double b1 = 1.0 / std::sqrt(9.0 * C), b2 = 1.0 / 24.0;   // fan-in 9C, 576
        for (int k = 0; k < C; ++k)
            for (size_t i = 0; i < n; ++i) {
                const float v = a[k * n + i];
                CHECK(std::isfinite(v));
                const double bound = i < (size_t)(64 * C * 9 + 64) ? b1 : (i < n - 65 ? b2 : 0.125);
                CHECK(std::fabs(v) <= bound);
            }
    }
    CHECK(n2f_param_count(0, &d, nullptr) == N2F_EINVAL);
    CHECK(n2f_init_params(1, &d, 0, nullptr) == N2F_EINVAL);
    return 0;
}

static int server_checks() {
    n2f_config d;
    n2f_config_default(&d);
    d.precision = N2F_BF16;
    size_t unit = 0;
    CHECK(n2f_workspace_bytes(512, 512, 1, &d, &unit) == N2F_OK);
    const size_t arena = 4 * unit;
    n2f_server* s = nullptr;
    CHECK(n2f_server_create(&s, &d, nullptr, arena, 4, 32, N2F_SERVER_SIMULATE) == N2F_OK);
    std::mt19937_64 rng(5);
    std::uniform_int_distribution<int> side(2, 1200), epochs(1, 30), ch(1, 3);
    const int n = 2000;
    int submitted = 0;
    std::set<long long> seen;
    std::vector<long long> ids(64);
    std::vector<int> st(64);
    std::set<long long> cancelled;
    for (int step = 0; step < 200000 && (int)seen.size() < n; ++step) {
        for (int k = 0; k < 3 && submitted < n; ++k, ++submitted) {
            const n2f_status r = n2f_server_submit(s, submitted, nullptr, nullptr, side(rng), side(rng), ch(rng),
                                                   epochs(rng), nullptr);
            if (r == N2F_ENOMEM) {   // could never fit: counted as done
                seen.insert(submitted);
                continue;
            }
            CHECK(r == N2F_OK);
            CHECK(n2f_server_submit(s, submitted, nullptr, nullptr, 8, 8, 1, 1, nullptr) == N2F_EINVAL);  // id in use
        }
        // every 37th request is cancelled a little after its submission
        // (queued or already active)
        if (submitted > 5 && (submitted - 5) % 37 == 0 && !seen.count(submitted - 5) &&
            !cancelled.count(submitted - 5)) {
            const n2f_status r = n2f_server_cancel(s, submitted - 5);
            CHECK(r == N2F_OK || r == N2F_EINVAL);   // EINVAL: it had already finished
            if (r == N2F_OK) cancelled.insert(submitted - 5);
        }
        int active = 0, queued = 0, got = 0;
        CHECK(n2f_server_step(s, 1, &active, &queued) == N2F_OK);
        CHECK(active <= 32);
        size_t used = 0, largest = 0;
        CHECK(n2f_server_memory(s, &used, &largest) == N2F_OK);
        CHECK(used <= arena && largest <= arena - used);
        CHECK(n2f_server_poll(s, ids.data(), st.data(), 64, &got) == N2F_OK);
        for (int i = 0; i < got; ++i) {
            CHECK(st[i] == (cancelled.count(ids[i]) ? N2F_ECANCELED : N2F_OK));
            CHECK(seen.insert(ids[i]).second);   // reported once
        }
    }
    CHECK((int)seen.size() == n);
    CHECK(!cancelled.empty());
    CHECK(n2f_server_cancel(s, 0) == N2F_EINVAL);   // long finished
    size_t used = 1, largest = 0;
    CHECK(n2f_server_memory(s, &used, &largest) == N2F_OK && used == 0 && largest == arena);
    CHECK(n2f_server_destroy(s) == N2F_OK);
    n2f_config ex = d;
    ex.exact_targets = 1;
    CHECK(n2f_server_create(&s, &ex, nullptr, arena, 1, 4, N2F_SERVER_SIMULATE) == N2F_EINVAL);
    CHECK(n2f_server_create(&s, &d, nullptr, arena, 1, 4, 0) == N2F_EINVAL);   // a real server needs an arena
    return 0;
}

static int argument_checks() {
    n2f_config d;
    n2f_config_default(&d);
    n2f_run* r = nullptr;
    CHECK(n2f_run_create(&r, nullptr, 8, 8, 1, &d, nullptr, 0, nullptr) == N2F_EINVAL && r == nullptr);
    CHECK(n2f_run_create(nullptr, nullptr, 8, 8, 1, &d, nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_train_step(nullptr, 0, 0) == N2F_EINVAL);
    CHECK(n2f_validate(nullptr, 0, nullptr, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_run_epochs(nullptr, 0, 1, nullptr) == N2F_EINVAL);
    CHECK(n2f_run_launch_epochs(nullptr, 0, 1) == N2F_EINVAL);
    CHECK(n2f_run_poll(nullptr, 0, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_result(nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_get_state(nullptr, 0, nullptr, nullptr, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_set_state(nullptr, 0, nullptr, nullptr, nullptr, 0) == N2F_EINVAL);
    CHECK(n2f_get_grad(nullptr, 0, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_debug_adam(nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_get_progress(nullptr, 0, nullptr, nullptr, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_get_history(nullptr, 0, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_get_lohi(nullptr, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_get_image(nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_run_set_clean(nullptr, nullptr) == N2F_EINVAL);
    size_t cb = 0;
    CHECK(n2f_checkpoint_bytes(nullptr, &cb) == N2F_EINVAL);
    CHECK(n2f_save_checkpoint(nullptr, 0, nullptr, 0) == N2F_EINVAL);
    CHECK(n2f_load_checkpoint(nullptr, 0, nullptr, 0) == N2F_EINVAL);
    CHECK(n2f_run_destroy(nullptr) == N2F_EINVAL);
    CHECK(n2f_denoise(nullptr, nullptr, 8, 8, 1, &d, nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_max_project(nullptr, 1, 1, nullptr, nullptr) == N2F_EINVAL);
    n2f_batch* b = nullptr;
    CHECK(n2f_batch_create(&b, 0, nullptr, nullptr, nullptr, nullptr, &d, nullptr, 0, 1, nullptr) == N2F_EINVAL);
    {   // grouped on more streams than the tables hold, and grouped FP32: refused before any device work
        const float* in1[1] = {reinterpret_cast<const float*>(256)};
        const int h1[1] = {8}, w1[1] = {8}, c1[1] = {1};
        n2f_config bf = d;
        bf.precision = N2F_BF16;
        CHECK(n2f_batch_create(&b, 1, in1, h1, w1, c1, &bf, reinterpret_cast<void*>(256), 1 << 30, -5, nullptr) ==
              N2F_EINVAL);
        n2f_config f32 = d;
        f32.precision = N2F_FP32;
        CHECK(n2f_batch_create(&b, 1, in1, h1, w1, c1, &f32, reinterpret_cast<void*>(256), 1 << 30, -2, nullptr) ==
              N2F_EINVAL);
        CHECK(n2f_group_grid_set(5, 0) == N2F_EINVAL);
        CHECK(n2f_group_grid_set(15, 256) == N2F_EINVAL);
        int gg = 0;
        CHECK(n2f_group_grid_get(-1, &gg) == N2F_EINVAL);
        CHECK(n2f_group_grid_get(5, nullptr) == N2F_EINVAL);
        CHECK(n2f_group_grid_get(5, &gg) == N2F_OK && gg >= 1);
    }
    CHECK(n2f_batch_add(nullptr, nullptr, 8, 8, 1, nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_batch_remove(nullptr, 0) == N2F_EINVAL);
    CHECK(n2f_server_cancel(nullptr, 0) == N2F_EINVAL);
    CHECK(n2f_batch_run(nullptr, 1, nullptr) == N2F_EINVAL);
    CHECK(n2f_batch_result(nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_batch_progress(nullptr, 0, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_batch_run_of(nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_batch_destroy(nullptr) == N2F_EINVAL);
    const int H[2] = {8, 1}, W[2] = {8, 8}, C[2] = {1, 1};
    size_t bb = 0;
    CHECK(n2f_batch_workspace_bytes(2, H, W, C, &d, &bb) == N2F_EINVAL);   // a 1-pixel-tall image
    CHECK(n2f_server_step(nullptr, 1, nullptr, nullptr) == N2F_EINVAL);
    CHECK(n2f_server_poll(nullptr, nullptr, nullptr, 0, nullptr) == N2F_EINVAL);
    CHECK(n2f_server_destroy(nullptr) == N2F_EINVAL);
    CHECK(n2f_profile_begin(0) == N2F_EINVAL);
    return 0;
}

int main() {
    if (config_checks() || plan_checks() || param_checks() || server_checks() || argument_checks()) return 1;
    std::printf("host checks passed\n");
    return 0;
}
