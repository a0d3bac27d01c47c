// Measured ceilings of the device, the denominators the SV and BFS kernels
// are judged against besides the published 8 TB/s: a streaming copy, and
// random 4-byte reads and random returning atomicMin on tables that live in
// one XCD's L2 (2 MiB, the size of a scale-24 vertex bitmap), in the
// Infinity Cache (64 MiB, a scale-24 parent array) and in HBM (4 GiB).  The
// random streams are counter-based (a 64-bit mix of the thread's counter), so
// they need no memory of their own; every thread keeps 8 accesses in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/cc.h"
#include "common.hpp"
#include "internal.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

namespace {

constexpr int kPeakBlock = 256;
constexpr int kInFlight = 8;
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // a bijective 64-bit finaliser (xor-shift and odd multiplies)
    z ^= z >> 31;
    z *= 0x7fb5d329728ea185ull;
    z ^= z >> 27;
    z *= 0x81dadef4bc2dd44dull;
    z ^= z >> 33;
    return z;
}

__global__ __launch_bounds__(kPeakBlock) void copy_kernel(const int4* __restrict__ src, int4* __restrict__ dst,
                                                          int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kPeakBlock;
    for (int64_t i = (int64_t)blockIdx.x * kPeakBlock + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// four 16-byte loads in flight per thread, then four stores; NT: the
// streaming (non-temporal) forms, which bypass the caches' allocation
template <bool NT>
__global__ __launch_bounds__(kPeakBlock) void copy4_kernel(const v4i* __restrict__ src, v4i* __restrict__ dst,
                                                           int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kPeakBlock;
    int64_t i = (int64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v4i x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = NT ? __builtin_nontemporal_load(src + i + k * stride) : src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (NT) __builtin_nontemporal_store(x[k], dst + i + k * stride);
            else dst[i + k * stride] = x[k];
        }
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

// streaming read: four 16-byte loads in flight per thread, xor-folded
template <bool NT>
__global__ __launch_bounds__(kPeakBlock) void read4_kernel(const v4i* __restrict__ src, int64_t n16,
                                                           int32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * kPeakBlock;
    int64_t i = (int64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    v4i acc = {0, 0, 0, 0};
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v4i x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = NT ? __builtin_nontemporal_load(src + i + k * stride) : src[i + k * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc ^= x[k];
    }
    for (; i < n16; i += stride) acc ^= src[i];
    sink[(int64_t)blockIdx.x * kPeakBlock + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

__global__ void fill_kernel(int32_t* __restrict__ p, int64_t n, int32_t value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = value;
}

// per thread: `rounds` rounds of kInFlight loads at mixed indexes below
// mask + 1 (a power of two); the xor of the values read goes to sink[]
__global__ __launch_bounds__(kPeakBlock) void gather_kernel(const int32_t* __restrict__ table, uint64_t mask,
                                                            int rounds, uint64_t seed, int32_t* __restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    int32_t acc = 0;
    for (int r = 0; r < rounds; ++r) {
        int32_t x[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k)
            x[k] = table[mix64(seed + (t * rounds + r) * kInFlight + k) & mask];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) acc ^= x[k];
    }
    sink[t] = acc;
}

// the same stream of indexes, each access an agent-scope atomicMin whose
// returned value is used, as a hook's is
__global__ __launch_bounds__(kPeakBlock) void atomic_kernel(int32_t* __restrict__ table, uint64_t mask, int rounds,
                                                            uint64_t seed, int32_t* __restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * kPeakBlock + threadIdx.x;
    int32_t acc = 0;
    for (int r = 0; r < rounds; ++r) {
        int32_t x[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
            const uint64_t h = mix64(seed + (t * rounds + r) * kInFlight + k);
            x[k] = atomic_min_agent(table + (h & mask), (int32_t)(h >> 40));
        }
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) acc ^= x[k];
    }
    sink[t] = acc;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes, const char* what) {
        hipError_t e = alloc_fault() ? hipErrorOutOfMemory : hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return hip_fail(e, what);
        }
        return CC_OK;
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_measure_peaks(cc_peaks* out, void* stream) {
    if (!out) return fail(CC_EINVAL, "NULL out");
    memset(out, 0, sizeof *out);
    hipStream_t s = (hipStream_t)stream;
    const size_t kCopy = (size_t)1 << 30;                 // bytes copied per launch
    const size_t kTables[3] = {(size_t)2 << 20, (size_t)64 << 20, (size_t)4 << 30};
    const int kBlocks = 256 * 16;                          // 16 workgroups per CU
    const int kRounds = 64;                                // 4096 * 256 * 64 * 8 = 2^29 accesses
    const int kReps = 5;
    DevBuf src, dst, table, sink;
    int rc;
    if ((rc = src.alloc(kCopy, "hipMalloc(peak copy source)"))) return rc;
    if ((rc = dst.alloc(kCopy, "hipMalloc(peak copy target)"))) return rc;
    if ((rc = table.alloc(kTables[2], "hipMalloc(peak table)"))) return rc;
    if ((rc = sink.alloc((size_t)kBlocks * kPeakBlock * sizeof(int32_t), "hipMalloc(peak sink)"))) return rc;
    Events ev;
    hipError_t e = create_timing_event(&ev.a);
    if (e == hipSuccess) e = create_timing_event(&ev.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    // best of kReps launches after one warm-up, in ms
    auto timed = [&](auto launch, double* best) -> int {
        *best = 1e30;
        for (int r = 0; r <= kReps; ++r) {
            hipError_t le = hipEventRecord(ev.a, s);
            if (le == hipSuccess) {
                launch(r);
                le = hipGetLastError();
            }
            if (le == hipSuccess) le = hipEventRecord(ev.b, s);
            if (le == hipSuccess) le = hipEventSynchronize(ev.b);
            float ms = 0.f;
            if (le == hipSuccess) le = hipEventElapsedTime(&ms, ev.a, ev.b);
            if (le != hipSuccess) return hip_fail(le, "peak measurement");
            if (r > 0) *best = std::min(*best, (double)ms);
        }
        return CC_OK;
    };
    fill_kernel<<<2048, 256, 0, s>>>((int32_t*)src.p, (int64_t)(kCopy / 4), 1);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "fill launch");
    double ms, best = 1e30;
    const int64_t n16 = (int64_t)(kCopy / 16);
    const int4* s4 = (const int4*)src.p;
    int4* d4 = (int4*)dst.p;
    const v4i* sv4 = (const v4i*)src.p;
    v4i* dv4 = (v4i*)dst.p;
    // the best of three copy forms: one 16-byte access per thread and step,
    // four in flight, four in flight with streaming hints
    if ((rc = timed([&](int) { copy_kernel<<<kBlocks, kPeakBlock, 0, s>>>(s4, d4, n16); }, &ms))) return rc;
    best = std::min(best, ms);
    if ((rc = timed([&](int) { copy4_kernel<false><<<kBlocks, kPeakBlock, 0, s>>>(sv4, dv4, n16); }, &ms))) return rc;
    best = std::min(best, ms);
    if ((rc = timed([&](int) { copy4_kernel<true><<<kBlocks, kPeakBlock, 0, s>>>(sv4, dv4, n16); }, &ms))) return rc;
    best = std::min(best, ms);
    out->copy_gbps = 2.0 * (double)kCopy / (best * 1e-3) / 1e9;
    out->copy_bytes = 2.0 * (double)kCopy;
    best = 1e30;
    if ((rc = timed([&](int) { read4_kernel<false><<<kBlocks, kPeakBlock, 0, s>>>(sv4, n16, (int32_t*)sink.p); },
                    &ms)))
        return rc;
    best = std::min(best, ms);
    if ((rc = timed([&](int) { read4_kernel<true><<<kBlocks, kPeakBlock, 0, s>>>(sv4, n16, (int32_t*)sink.p); },
                    &ms)))
        return rc;
    best = std::min(best, ms);
    out->read_gbps = (double)kCopy / (best * 1e-3) / 1e9;
    const double accesses = (double)kBlocks * kPeakBlock * kRounds * kInFlight;
    for (int k = 0; k < 3; ++k) {
        const uint64_t mask = kTables[k] / 4 - 1;
        out->table_bytes[k] = (int64_t)kTables[k];
        fill_kernel<<<2048, 256, 0, s>>>((int32_t*)table.p, (int64_t)(kTables[k] / 4), INT32_MAX);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "fill launch");
        if ((rc = timed([&](int r) {
                 gather_kernel<<<kBlocks, kPeakBlock, 0, s>>>((const int32_t*)table.p, mask, kRounds,
                                                              0x9e3779b97f4a7c15ull * (uint64_t)(r + 1),
                                                              (int32_t*)sink.p);
             }, &ms)))
            return rc;
        out->gather_gps[k] = accesses / (ms * 1e-3) / 1e9;
        if ((rc = timed([&](int r) {
                 atomic_kernel<<<kBlocks, kPeakBlock, 0, s>>>((int32_t*)table.p, mask, kRounds,
                                                              0xd1b54a32d192ed03ull * (uint64_t)(r + 1),
                                                              (int32_t*)sink.p);
             }, &ms)))
            return rc;
        out->atomic_gps[k] = accesses / (ms * 1e-3) / 1e9;
    }
    out->accesses = accesses;
    e = hipStreamSynchronize(s);
    return e == hipSuccess ? CC_OK : hip_fail(e, "hipStreamSynchronize");
}
