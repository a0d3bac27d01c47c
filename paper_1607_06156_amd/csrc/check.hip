// Debug checks of the labelling invariants, run on the device:
//  - during SV: every parent link points to an id no larger than the vertex
//    (hooks only ever link a root under a smaller id, Section III-A.2, and a
//    shortcut only moves a link further down), and stays inside [0, n);
//  - on a finished labelling: I1, the two ends of every edge carry the same
//    label, and I2, labels[x] <= x and labels[labels[x]] == labels[x] (the
//    label is a vertex of the component that labels itself).
// Both catch a lost or misdirected link; neither can see two components that
// were merged into one (the oracle comparison of the tests does).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "../../include/cc.h"
#include "common.hpp"
#include "internal.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

namespace {

constexpr int kCheckBlocks = 2048;
constexpr unsigned long long kNone = ~0ull;

__device__ __forceinline__ void reduce_report(unsigned long long bad, unsigned long long first,
                                              unsigned long long* cnt, unsigned long long* where) {
    for (int o = 32; o > 0; o >>= 1) {
        bad += __shfl_xor(bad, o);
        const unsigned long long f = __shfl_xor(first, o);
        first = f < first ? f : first;
    }
    if (lane_id() == 0 && bad) {
        atomic_add_agent(cnt, bad);
        __hip_atomic_fetch_min(where, first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// out[0]: vertices whose link leaves [0, x]; out[1]: the smallest of them
__global__ __launch_bounds__(kBlock) void check_parent_kernel(const int32_t* __restrict__ parent, int32_t n,
                                                              unsigned long long* out) {
    unsigned long long bad = 0, first = kNone;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += stride) {
        const int32_t p = parent[x];
        if (p < 0 || (int64_t)p > x) {
            ++bad;
            if ((unsigned long long)x < first) first = (unsigned long long)x;
        }
    }
    reduce_report(bad, first, out, out + 1);
}

// out[0..1]: edges whose ends carry different labels (I1) and the first;
// out[2..3]: vertices breaking I2 and the first; out[4..5]: edges with an
// end outside [0, n) and the first
__global__ __launch_bounds__(kBlock) void check_labels_kernel(const int32_t* __restrict__ u,
                                                              const int32_t* __restrict__ v, int64_t m,
                                                              const int32_t* __restrict__ labels, int32_t n,
                                                              unsigned long long* out) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long b1 = 0, f1 = kNone, br = 0, fr = kNone;
    for (int64_t i = t0; i < m; i += stride) {
        const int32_t a = u[i], b = v[i];
        if (a < 0 || a >= n || b < 0 || b >= n) {
            ++br;
            if ((unsigned long long)i < fr) fr = (unsigned long long)i;
        } else if (labels[a] != labels[b]) {
            ++b1;
            if ((unsigned long long)i < f1) f1 = (unsigned long long)i;
        }
    }
    reduce_report(b1, f1, out, out + 1);
    reduce_report(br, fr, out + 4, out + 5);
    unsigned long long b2 = 0, f2 = kNone;
    for (int64_t x = t0; x < n; x += stride) {
        const int32_t l = labels[x];
        const bool ok = l >= 0 && (int64_t)l <= x && labels[l] == l;
        if (!ok) {
            ++b2;
            if ((unsigned long long)x < f2) f2 = (unsigned long long)x;
        }
    }
    reduce_report(b2, f2, out + 2, out + 3);
}

unsigned grid_for(int64_t items) {
    const int64_t b = (items + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kCheckBlocks));
}

// out[2k] = 0 (counts), out[2k + 1] = kNone (first offenders)
__global__ void check_init_kernel(unsigned long long* out, int words) {
    const int i = threadIdx.x;
    if (i < words) out[i] = (i & 1) ? kNone : 0ull;
}

int readback(hipStream_t s, unsigned long long* host, const unsigned long long* dev, int words) {
    hipError_t e = hipMemcpyAsync(host, dev, words * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? CC_OK : hip_fail(e, "check readback");
}

}  // namespace

int check_enabled(const cc_options& opt) {
    if (opt.check) return 1;
    const char* env = getenv("CCMI_CHECK");
    return env && env[0] && env[0] != '0' ? 1 : 0;
}

int check_parent(Workspace& ws, hipStream_t s, const int32_t* parent, int32_t n, int pass) {
    void* p;
    unsigned long long* host;
    int rc;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &p))) return rc;
    if ((rc = ws.pinned((void**)&host))) return rc;
    unsigned long long* out = (unsigned long long*)p + kCheckWords;
    check_init_kernel<<<1, 64, 0, s>>>(out, 2);
    check_parent_kernel<<<grid_for(n), kBlock, 0, s>>>(parent, n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "check_parent launch");
    if ((rc = readback(s, host, out, 2))) return rc;
    if (host[0])
        return fail(CC_EINTERNAL, "check: after SV pass %d, %llu vertices link outside [0, x] (first: vertex %llu)",
                    pass, host[0], host[1]);
    return CC_OK;
}

int check_labels(Workspace& ws, hipStream_t s, const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                 const int32_t* labels, int64_t bad[3], int64_t first[3]) {
    void* p;
    unsigned long long* host;
    int rc;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &p))) return rc;
    if ((rc = ws.pinned((void**)&host))) return rc;
    unsigned long long* out = (unsigned long long*)p + kCheckWords;
    check_init_kernel<<<1, 64, 0, s>>>(out, 6);
    check_labels_kernel<<<grid_for(std::max<int64_t>(m, n)), kBlock, 0, s>>>(u, v, m, labels, n, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "check_labels launch");
    if ((rc = readback(s, host, out, 6))) return rc;
    for (int k = 0; k < 3; ++k) {
        bad[k] = (int64_t)host[2 * k];
        first[k] = host[2 * k] ? (int64_t)host[2 * k + 1] : -1;
    }
    return CC_OK;
}

int check_result(Workspace& ws, hipStream_t s, const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                 const int32_t* labels) {
    int64_t bad[3], first[3];
    int rc = check_labels(ws, s, u, v, m, n, labels, bad, first);
    if (rc) return rc;
    if (bad[0] || bad[1] || bad[2])
        return fail(CC_EINTERNAL,
                    "check: %lld edges with differently labelled ends (first: edge %lld), %lld vertices whose "
                    "label is above them or not its own label (first: vertex %lld), %lld edges out of range",
                    (long long)bad[0], (long long)first[0], (long long)bad[1], (long long)first[1],
                    (long long)bad[2]);
    return CC_OK;
}

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_check_labels(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const int32_t* labels,
                           void* stream, int64_t* bad) {
    if (!bad) return fail(CC_EINVAL, "NULL bad");
    bad[0] = bad[1] = bad[2] = 0;
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size (m=%lld, n=%d)", (long long)m, n);
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge array");
    if (n > 0 && !labels) return fail(CC_EINVAL, "NULL labels");
    if (m > 0 && n == 0) {
        bad[2] = m;
        return CC_OK;
    }
    if (n == 0) return CC_OK;
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(ws->mu);
    int64_t first[3];
    return check_labels(*ws, (hipStream_t)stream, u, v, m, n, labels, bad, first);
}
