// Arbitrary 64-bit vertex ids (Section III-B, relabelling before the BFS;
// Section V: every vertex id is a 64-bit integer, as k-mers are).
//
// The paper relabels the ids of the graph to [0, |V|) with sorts.  Here the
// distinct endpoint ids are gathered in a device hash table (open addressing,
// linear probing, 64-bit compare-and-swap), the occupied slots are numbered
// by a device-wide scan, which gives every distinct id a compact id in
// [0, n), and the edges are rewritten in compact ids.  The 32-bit path then
// labels the compact graph (label = smallest compact id of the component),
// and the labels are mapped back: every component's smallest original id is
// found with a 64-bit atomicMin into the entry of its compact root, and every
// vertex copies its root's entry.  The output lists each distinct id once
// with the smallest original id of its component.
//
// Every 64-bit value is a valid id.  The table marks an empty slot with
// INT64_MIN; the id INT64_MIN itself gets the extra slot after the table.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/cc.h"
#include "internal.hpp"
#include "scan.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

constexpr int64_t kEmpty64 = INT64_MIN;

// 64-bit finaliser of MurmurHash3 (Appleby): spreads the ids over the table
__device__ __forceinline__ uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__global__ __launch_bounds__(kBlock) void h64_clear_kernel(int64_t* __restrict__ keys, int64_t cap,
                                                           unsigned long long* __restrict__ flags) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < cap; i += stride) keys[i] = kEmpty64;
    if (blockIdx.x == 0 && threadIdx.x < 4) flags[threadIdx.x] = 0;
}

// Slot of id, inserting it if absent.  Keys never change once set, so a
// plain load that sees another key is final; a load that sees an empty slot
// is confirmed by the compare-and-swap, which returns the slot's true key.
// The walk is bounded by the table size: a full table sets flags[1].
__device__ __forceinline__ uint32_t h64_insert(int64_t* keys, uint64_t mask, int64_t id,
                                               unsigned long long* flags) {
    if (id == kEmpty64) {
        if (__hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            __hip_atomic_store(&flags[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return (uint32_t)(mask + 1);   // the extra slot
    }
    uint64_t h = mix64((uint64_t)id) & mask;
    for (uint64_t t = 0; t <= mask; ++t) {
        const int64_t k = keys[h];
        if (k == id) return (uint32_t)h;
        if (k == kEmpty64) {
            unsigned long long expected = (unsigned long long)kEmpty64;
            __hip_atomic_compare_exchange_strong((unsigned long long*)&keys[h], &expected, (unsigned long long)id,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int64_t)expected == kEmpty64 || (int64_t)expected == id) return (uint32_t)h;
        }
        h = (h + 1) & mask;
    }
    atomic_add_agent(&flags[1], 1ull);
    return 0;
}

// slot of every endpoint: su[i] = slot(u[i]), sv[i] = slot(v[i])
__global__ __launch_bounds__(kBlock) void h64_insert_kernel(const int64_t* __restrict__ u,
                                                            const int64_t* __restrict__ v, int64_t m,
                                                            int64_t* keys, uint64_t mask, uint32_t* __restrict__ su,
                                                            uint32_t* __restrict__ sv,
                                                            unsigned long long* flags) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const int64_t a = u[i], b = v[i];
        su[i] = h64_insert(keys, mask, a, flags);
        sv[i] = h64_insert(keys, mask, b, flags);
    }
}

// edges in compact ids, in place: s[i] <- cid[s[i]]
__global__ __launch_bounds__(kBlock) void h64_map_kernel(uint32_t* __restrict__ su, uint32_t* __restrict__ sv,
                                                         int64_t m, const uint32_t* __restrict__ cid) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        su[i] = cid[su[i]];
        sv[i] = cid[sv[i]];
    }
}

__global__ __launch_bounds__(kBlock) void l64_init_kernel(int64_t* __restrict__ lab, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += stride) lab[x] = INT64_MAX;
}

// lab[root of x] = min over the component of the original ids
__global__ __launch_bounds__(kBlock) void l64_min_kernel(const int32_t* __restrict__ lab32,
                                                         const int64_t* __restrict__ ids, int64_t n,
                                                         int64_t* lab) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += stride)
        __hip_atomic_fetch_min(&lab[lab32[x]], ids[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// every vertex that is not its component's compact root copies the root's
// entry (roots keep theirs, so no entry that is read is written)
__global__ __launch_bounds__(kBlock) void l64_copy_kernel(const int32_t* __restrict__ lab32, int64_t n,
                                                          int64_t* lab) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += stride) {
        const int32_t r = lab32[x];
        if (r != (int32_t)x) lab[x] = lab[r];
    }
}

static int grid_of(int64_t items) {
    int64_t g = (items + 4 * kBlock - 1) / (4 * kBlock);
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

struct SlotCount {
    const int64_t* keys;
    int64_t cap;
    const unsigned long long* flags;
    __device__ uint32_t operator()(int64_t s) const {
        return s < cap ? (uint32_t)(keys[s] != kEmpty64) : (uint32_t)(flags[0] != 0);
    }
};

struct SlotEmit {
    const int64_t* keys;
    int64_t cap;
    uint32_t* cid;
    int64_t* ids;
    int64_t n_max;
    __device__ void operator()(int64_t s, uint32_t pre, uint32_t c) const {
        if (!c) return;
        cid[s] = pre;
        if ((int64_t)pre < n_max) ids[pre] = s < cap ? keys[s] : kEmpty64;
    }
};

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_label64_ex(const int64_t* u, const int64_t* v, int64_t m, int64_t n_max, int64_t* ids,
                         int64_t* labels, int64_t* n_out, void* stream, const cc_options* opt_in, cc_stats* stats) {
    if (!n_out) return fail(CC_EINVAL, "NULL n_out");
    *n_out = 0;
    if (m < 0) return fail(CC_EINVAL, "negative m");
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge array");
    if (n_max <= 0) n_max = 2 * m;
    if (n_max > ((int64_t)1 << 30))
        return fail(CC_EINVAL, "n_max = %lld distinct ids is above 2^30 (give a smaller bound)", (long long)n_max);
    if (m > 0 && (!ids || !labels)) return fail(CC_EINVAL, "NULL output");
    cc_options opt;
    if (opt_in) opt = *opt_in; else cc_default_options(&opt);
    if (opt.workspace) return fail(CC_EINVAL, "cc_label64 takes no caller workspace");
    if (opt.route < CC_ROUTE_AUTO || opt.route > CC_ROUTE_SV_THETA) return fail(CC_EINVAL, "bad route %d", opt.route);
    if (opt.max_passes < 0) return fail(CC_EINVAL, "negative max_passes");
    if (stats) memset(stats, 0, sizeof *stats);
    if (m == 0) return CC_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::unique_lock<std::mutex> lk(ws->mu);

    int64_t cap = 1024;
    while (cap < 2 * n_max) cap <<= 1;
    const uint64_t mask = (uint64_t)cap - 1;
    void *pk, *pc, *pe, *pf, *pb;
    if ((rc = ws->get(WS_R64_KEYS, (size_t)cap * sizeof(int64_t), &pk))) return rc;
    if ((rc = ws->get(WS_R64_CID, (size_t)(cap + 1) * sizeof(uint32_t), &pc))) return rc;
    const size_t half = ((size_t)m * sizeof(uint32_t) + 255) & ~(size_t)255;
    if ((rc = ws->get(WS_R64_EDGES, 2 * half, &pe))) return rc;
    if ((rc = ws->get(WS_R64_FLAGS, 8 * sizeof(unsigned long long), &pf))) return rc;
    if ((rc = ws->get(WS_R64_SCAN, (size_t)scan_tiles(cap + 1) * sizeof(uint32_t), &pb))) return rc;
    int64_t* keys = (int64_t*)pk;
    uint32_t* cid = (uint32_t*)pc;
    uint32_t* su = (uint32_t*)pe;
    uint32_t* sv = (uint32_t*)((char*)pe + half);
    unsigned long long* flags = (unsigned long long*)pf;   // [0] INT64_MIN seen, [1] table full, [2] distinct ids
    unsigned long long* host;
    if ((rc = ws->pinned((void**)&host))) return rc;

    h64_clear_kernel<<<grid_of(cap), kBlock, 0, s>>>(keys, cap, flags);
    h64_insert_kernel<<<grid_of(m), kBlock, 0, s>>>(u, v, m, keys, mask, su, sv, flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "relabel insert launch");
    SlotCount cnt{keys, cap, flags};
    SlotEmit emit{keys, cap, cid, ids, n_max};
    if ((e = device_scan(cnt, emit, cap + 1, (uint32_t*)pb, flags + 2, s)) != hipSuccess)
        return hip_fail(e, "relabel scan launch");
    if ((e = hipMemcpyAsync(host, flags, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "relabel readback");
    if (host[1]) return fail(CC_EINTERNAL, "hash table of %lld slots overflowed", (long long)cap);
    const int64_t n = (int64_t)host[2];
    if (n > n_max) return fail(CC_EINVAL, "%lld distinct ids, more than n_max = %lld", (long long)n, (long long)n_max);
    h64_map_kernel<<<grid_of(m), kBlock, 0, s>>>(su, sv, m, cid);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "relabel map launch");

    // the compact graph through the 32-bit path; its labels in WS_R64_KEYS,
    // whose table is no longer needed (n <= cap / 2 entries of 4 bytes)
    int32_t* lab32 = (int32_t*)keys;
    Call c;
    c.ws = ws;
    c.stream = s;
    c.u = (const int32_t*)su;
    c.v = (const int32_t*)sv;
    c.m = m;
    c.n = (int32_t)n;
    c.parent = lab32;
    c.stats = stats;
    c.opt = opt;
    if (c.opt.tau <= 0) c.opt.tau = 0.05;
    if (c.opt.theta < 1) c.opt.theta = 8.0;
    Timer tm(stats != nullptr, s);
    c.timer = &tm;
    if (stats) {
        stats->route = -1;
        stats->bfs_seed = -1;
        stats->bfs_label = -1;
        stats->max_degree = -1;
    }
    if ((rc = run_label(c))) return rc;
    l64_init_kernel<<<grid_of(n), kBlock, 0, s>>>(labels, n);
    l64_min_kernel<<<grid_of(n), kBlock, 0, s>>>(lab32, ids, n, labels);
    l64_copy_kernel<<<grid_of(n), kBlock, 0, s>>>(lab32, n, labels);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "label map-back launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *n_out = n;
    return CC_OK;
}

CC_API int cc_label64(const int64_t* u, const int64_t* v, int64_t m, int64_t n_max, int64_t* ids, int64_t* labels,
                      int64_t* n_out, void* stream) {
    return cc_label64_ex(u, v, m, n_max, ids, labels, n_out, stream, nullptr, nullptr);
}
