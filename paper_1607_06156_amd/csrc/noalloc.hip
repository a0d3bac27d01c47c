// cc_label_noalloc: the plain SV route of cc_label with no allocation at all.
//
// The call's device scratch (the active-edge segment buffers, the hooked-root
// lists, the per-segment counters and the pass totals) lives in one
// file-scope device array of fixed size, `scratch`, which the code object
// brings with it: every GPU the library runs on holds its own copy from
// load time until the process ends.  Host code never passes the array's name
// to a kernel or a copy (in host code it only names a host-side stand-in):
// the device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and used from then on.  Readbacks go through a buffer
// on the calling thread's stack.  Calls that overlap on one GPU share that
// GPU's array and race; the caller must not overlap them.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "../../include/cc.h"
#include "internal.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

static __device__ __align__(256) unsigned char scratch[CC_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::unordered_map<int, void*> g_scratch_dev;   // device -> address of its copy

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with it current) and kept.
static int scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it != g_scratch_dev.end()) {
        *out = it->second;
        return CC_OK;
    }
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev.emplace(dev, ptr);
    *out = ptr;
    return CC_OK;
}

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_label_noalloc(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream) {
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size (m=%lld, n=%d)", (long long)m, n);
    if (m > 0 && n == 0) return fail(CC_EINVAL, "edges given for an empty vertex set");
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge array");
    if (n > 0 && !labels) return fail(CC_EINVAL, "NULL labels");
    Workspace ws;
    const size_t need = workspace_bound(m, n, true, ws.bound);
    if (need > (size_t)CC_NOALLOC_SCRATCH_BYTES)
        return fail(CC_EINVAL, "%lld edges need %zu bytes of scratch, more than the fixed %d", (long long)m, need,
                    (int)CC_NOALLOC_SCRATCH_BYTES);
    if (n == 0) return CC_OK;
    int rc;
    hipError_t e = hipGetDevice(&ws.device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    void* base = nullptr;
    if ((rc = scratch_address(ws.device, &base))) return rc;
    // readbacks of the SV loop: a few words of counters
    alignas(64) unsigned long long stage[64];
    ws.mode = Workspace::kArena;
    ws.arena = (char*)base;
    ws.arena_bytes = CC_NOALLOC_SCRATCH_BYTES;
    ws.host = stage;
    ws.host_external = true;

    Call c;
    c.ws = &ws;
    c.stream = (hipStream_t)stream;
    c.n = n;
    c.m = m;
    c.u = u;
    c.v = v;
    c.parent = labels;
    cc_default_options(&c.opt);
    c.opt.route = CC_ROUTE_SV;
    Timer tm(false, c.stream);
    c.timer = &tm;
    if ((rc = run_label(c))) return rc;
    e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return CC_OK;
}
