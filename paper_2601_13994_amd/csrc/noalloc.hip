// Allocation-free shared-pattern solves for callers that cannot allocate
// device memory during a call (tight serving loops, harnesses that forbid
// hipMalloc).  The solver's workspace -- per-system state records, block
// partials, work vectors and the per-solve diagonal-major copies -- lives in
// one file-scope device array instead of the handle's allocation.
//
// Every device that loads this library holds its own copy of `scratch` until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol); hsla_create looks up this
// device's address with hipGetSymbolAddress once per device, and the entry
// point hands that address to the same kernels hsla_solve_batched runs.
#include <mutex>

#include "common.h"

namespace hsla {
namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hsla_status scratch_init(hsla_handle *h) {
    if (h->device < 0 || h->device >= kMaxDevices)
        return set_error(h, HSLA_ERR_INVALID_ARG, "device %d beyond the scratch table", h->device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[h->device]) return HSLA_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return set_error(h, HSLA_ERR_HIP, "scratch address on device %d: %s", h->device, hipGetErrorString(e));
    g_scratch_ptr[h->device] = ptr;
    return HSLA_OK;
}

static void *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

}  // namespace hsla

extern "C" hsla_status hsla_solve_noalloc(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                                          const double *d_b, double *d_x, const hsla_opts *opts, hsla_info *infos,
                                          void *stream) {
    using namespace hsla;
    if (!h) return HSLA_ERR_INVALID_ARG;
    if (B < 0 || B > kNoAllocMaxSystems)
        return set_error(h, HSLA_ERR_INVALID_ARG, "batch of %d systems; the allocation-free solve takes 0..%d", B,
                         kNoAllocMaxSystems);
    hsla_opts o;
    if (opts)
        o = *opts;
    else
        hsla_opts_default(&o);
    if (o.profile) return set_error(h, HSLA_ERR_INVALID_ARG, "profile mode creates events; not allocation-free");
    // instantiating a graph allocates: iterations are launched one by one
    o.use_graph = 0;
    void *ptr = scratch_of(h->device);
    if (!ptr) {
        // hsla_create's lookup failed: try once more with the device current
        HSLA_HIP(h, hipSetDevice(h->device));
        const hsla_status se = scratch_init(h);
        if (se != HSLA_OK) return se;
        ptr = scratch_of(h->device);
    }
    if (h->h_state_cap < (size_t)B)
        return set_error(h, HSLA_ERR_INTERNAL, "host state mirror holds %zu systems", h->h_state_cap);
    // run the ordinary solve on the scratch array; the handle's own
    // workspace is put back afterwards, whatever the outcome
    void *own = h->ws;
    const size_t own_bytes = h->ws_bytes;
    h->ws = ptr;
    h->ws_bytes = kNoAllocScratchBytes;
    h->ws_fixed = true;
    const hsla_status st = solve_entry(h, p, B, d_values, d_b, d_x, &o, infos, (hipStream_t)stream);
    h->ws = own;
    h->ws_bytes = own_bytes;
    h->ws_fixed = false;
    return st;
}
