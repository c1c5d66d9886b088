// The allocation-free query entry point: one query whose whole device
// workspace (K block, optional K .* M, row shifts and iterate, parameter
// block) lives in a fixed device array, so the call makes no device or pinned
// host allocation and can be used where allocating is not allowed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "wmd_corpus.h"

namespace wmd {
constexpr size_t kScratchBytes = WMD_NOALLOC_SCRATCH_BYTES;
}  // namespace wmd

// Held by every device the library runs on until the process ends.  Host code
// never uses this name as an address: each device's copy is reached through
// the pointer resolved by scratch_setup.
static __device__ __align__(256) char scratch[wmd::kScratchBytes];

namespace wmd {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};   // the array's address on each device, once resolved
}  // namespace

int scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(WMD_EINVAL, "device ordinal %d above the library's limit", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return WMD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "scratch: symbol address");
    g_scratch[dev] = static_cast<char*>(p);
    return WMD_OK;
}

static char* scratch_of(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
}

}  // namespace wmd

using namespace wmd;

extern "C" int wmd_query_noalloc(wmd_corpus* c, const int32_t* qids, const float* qweights, int32_t n,
                                 float lambda, int32_t iters, const wmd_query_options* opt, double* dev_dist,
                                 double* dev_resid, void* stream) {
    if (!c || !dev_dist) return fail(WMD_EINVAL, "query: null corpus or output");
    wmd_query_options o;
    int rc = check_query_options(opt, &o);
    if (rc) return rc;
    std::vector<PlannedQuery> qs(1);
    if ((rc = plan_query(c, qids, qweights, n, lambda, iters, o.precision == WMD_DIST_BF16, &qs[0]))) return rc;
    const Layout L = make_layout(c, qs, o, dev_resid != nullptr, false);
    if (L.device_bytes() > kScratchBytes)
        return fail(WMD_EINVAL, "query: needs %zu bytes of workspace, the fixed scratch holds %zu", L.device_bytes(),
                    kScratchBytes);
    if (L.pbytes > (size_t)kUploadMaxBytes)
        return fail(WMD_EINVAL, "query: parameter block of %zu bytes exceeds the %d bytes that travel as kernel "
                                "arguments", L.pbytes, kUploadMaxBytes);
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard guard(c->dc.device);
    if (!guard.ok()) return fail(WMD_EDEVICE, "query: cannot select device");
    char* base = scratch_of(c->dc.device);
    if (!base) return fail(WMD_EDEVICE, "query: scratch not set up on device %d", c->dc.device);
    // a workspace carved from the scratch array: no event, no pinned memory;
    // the parameter block travels as kernel arguments, so the staging ring
    // (which would allocate pinned memory) is never touched
    Workspace w;
    carve_workspace(w, base, L);
    Staging unused;
    return enqueue_queries(c, qs, o, dev_dist, dev_resid, (hipStream_t)stream, false, w, unused, false);
}
