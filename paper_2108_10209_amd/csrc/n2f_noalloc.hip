// One-shot denoise for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Same computation as n2f_denoise, with the run's workspace in
// a fixed device array of this library instead of a caller buffer.
//
// The array holds kScratchBytes on every device the library runs on, for
// the life of the process.  Host code must not use its name as a device
// address: on first use per device (with that device current) its address
// is looked up once with hipGetSymbolAddress and kept; only that address is
// passed on.  Calls on one device share the array: they must not overlap
// (each call synchronises its stream before it returns).  Everything a run
// reads is written by the run itself first (n2f_run_create clears its
// state, moments, sums and counters), so one call's leftovers never leak
// into the next.
#include "n2f.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "n2f_internal.h"

namespace {

constexpr size_t kScratchBytes = N2F_NOALLOC_MAX_BYTES;   // per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch[kMaxDevices];
hipError_t g_lookup[kMaxDevices];
std::once_flag g_once[kMaxDevices];

}  // namespace

extern "C" n2f_status n2f_denoise_noalloc(const float* d_in, float* d_out, int H, int W, int C,
                                          const n2f_config* cfg, hipStream_t stream) {
    if (!d_in || !d_out || !cfg) {
        n2f::set_last_error("input, output or config is NULL");
        return N2F_EINVAL;
    }
    if (n2f::profiling_on()) {   // the kernel timer creates HIP events
        n2f::set_last_error("kernel timing is on (n2f_profile_begin): call n2f_profile_end first");
        return N2F_ESTATE;
    }
    size_t need = 0;
    n2f_status s = n2f_workspace_bytes(H, W, C, cfg, &need);
    if (s != N2F_OK) return s;
    if (need > kScratchBytes) {
        n2f::set_last_error("image needs a " + std::to_string(need) + "-byte workspace; the fixed device array holds " +
                            std::to_string(kScratchBytes) + " bytes (use n2f_denoise with a caller workspace)");
        return N2F_ENOMEM;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        n2f::set_last_error("no usable current device");
        return N2F_EDEVICE;
    }
    std::call_once(g_once[dev], [dev] { g_lookup[dev] = hipGetSymbolAddress(&g_scratch[dev], HIP_SYMBOL(scratch)); });
    if (g_lookup[dev] != hipSuccess || !g_scratch[dev]) {
        n2f::set_last_error(std::string("device address of the fixed workspace: ") + hipGetErrorString(g_lookup[dev]));
        return N2F_EDEVICE;
    }
    // direct launches: instantiating a graph may allocate device memory
    n2f_config c = *cfg;
    c.use_graph = 0;
    return n2f_denoise(d_in, d_out, H, W, C, &c, g_scratch[dev], kScratchBytes, stream);
}
