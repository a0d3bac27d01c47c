// Algorithm 1 as the paper runs it: the tuple array and its sorts
// (Section III-A.2, with the parallel sorts of Section III-A.3), on the GPU.
// This is the ablation beside the atomic-hooking SV of sv.hip: the same
// labels, computed by grouping tuples with sorts, so the share of the time
// the sorts take can be measured (Section V, Performance Anatomy).
//
// The array A holds tuples <p, q, r> (r a vertex, p its partition, q the
// candidate partition), stored as int4 {p, q, r, temporary}.  A_0 has
// <x, _, x> per vertex and <u, _, v>, <v, _, u> per edge.  An iteration:
//   1. sort by (r, p): the first tuple of each vertex bucket VB(u) holds
//      u_min = min M(u); every tuple of the bucket takes it as q;
//   2. sort by (p, q): the first tuple of each partition bucket PB(p) holds
//      p_min = min C(p); every tuple of the bucket moves to partition p_min;
//   3. a temporary tuple <p_min, _, p_min> per partition of the result;
//   4. steps 1 and 2 again with the temporary tuples (pointer doubling, Fig.
//      "doubling"), then the temporary tuples are erased.
// The loop ends when no partition changed in either step 2.  The label of u
// is p of any tuple <p, q, u>.
// With exclusion (Section III-A.4), after step 2 a tuple is potentially
// completed when its vertex bucket holds a single partition (the bucket's
// largest p equals its smallest); a partition all of whose tuples are
// potentially completed, and which did not move, is complete: its tuples get
// their labels and leave the array before step 3.  Without it every
// iteration sorts the whole array.
//
// The sorts are least-significant-digit radix sorts on the two 32-bit fields
// of the key (8-bit digits over the bits that ids below n use): per digit a
// histogram of each 4096-tuple tile, a device-wide scan of the counts in
// digit-major order, and a stable scatter.  A bucket's first tuple then
// writes its value into a per-vertex slot, from which the bucket's other
// tuples read it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "../../include/cc.h"
#include "internal.hpp"
#include "scan.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsRounds = 16;                                  // 64-tuple rounds per wave
constexpr int64_t kRsTile = (int64_t)kRsThreads * kRsRounds;   // tuples per tile
constexpr int32_t kNone = INT32_MAX;                           // the "_" of a tuple
// tuple.w flags
constexpr int32_t kTmp = 1;    // a temporary tuple
constexpr int32_t kPot = 2;    // potentially completed (its vertex bucket holds one partition)
constexpr int32_t kDone = 4;   // its partition is complete: leaves the array

// composite key of a tuple: by (r, p) when by_p is false, by (p, q) when true
__device__ __forceinline__ uint64_t tuple_key(const int4& t, bool by_p, int bits) {
    const uint32_t hi = (uint32_t)(by_p ? t.x : t.z);
    const uint32_t lo = (uint32_t)(by_p ? t.y : t.x);
    return ((uint64_t)hi << bits) | lo;
}

// counts[d * nt + tile] = tuples of the tile whose digit is d
__global__ __launch_bounds__(kRsThreads) void rs_hist_kernel(const int4* __restrict__ in, int64_t T, bool by_p,
                                                             int bits, int shift, int64_t nt,
                                                             uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsRounds; ++k) {
        const int64_t i = base + (int64_t)k * kRsThreads + threadIdx.x;
        if (i < T) atomicAdd(&h[(tuple_key(in[i], by_p, bits) >> shift) & 0xff], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nt + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile.  Wave w takes the tile's tuples
// [w * 1024, (w + 1) * 1024) in 16 rounds of 64; within a round, lanes with
// the same digit find each other with 8 ballots, so each tuple's rank among
// the wave's tuples of its digit (earlier rounds, then lower lanes) needs no
// barrier.  The waves' counts are then scanned per digit in wave order, and
// each tuple goes to offs[d * nt + tile] + (earlier waves' count of d) + rank.
__global__ __launch_bounds__(kRsThreads) void rs_scatter_kernel(const int4* __restrict__ in, int4* __restrict__ out,
                                                                int64_t T, bool by_p, int bits, int shift, int64_t nt,
                                                                const uint32_t* __restrict__ offs) {
    __shared__ uint32_t wcnt[kRsWaves][256];
    const int w = threadIdx.x >> 6, lane = lane_id();
    for (int d = threadIdx.x; d < 256 * kRsWaves; d += kRsThreads) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * (kRsRounds * 64);
    const uint64_t below = (1ull << lane) - 1ull;
    int4 t[kRsRounds];
    uint32_t dig[kRsRounds], rank[kRsRounds];
#pragma unroll
    for (int k = 0; k < kRsRounds; ++k) {
        const int64_t i = base + (int64_t)k * 64 + lane;
        const bool ok = i < T;
        if (ok) t[k] = in[i];
        const uint32_t d = ok ? (uint32_t)((tuple_key(t[k], by_p, bits) >> shift) & 0xff) : 256u;
        uint64_t peers = ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t m = ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        dig[k] = d;
        uint32_t r = 0;
        if (ok) r = wcnt[w][d] + (uint32_t)__popcll(peers & below);
        rank[k] = r;
        // the lowest lane of each digit adds the round's count after every
        // lane of the wave has read the old one
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers & below) == 0) wcnt[w][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int x = 0; x < kRsWaves; ++x) {
            const uint32_t c = wcnt[x][d];
            wcnt[x][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRsRounds; ++k) {
        const uint32_t d = dig[k];
        if (d < 256u) out[(int64_t)offs[(int64_t)d * nt + blockIdx.x] + wcnt[w][d] + rank[k]] = t[k];
    }
}

// first tuple of each bucket (sorted by key hi, then lo): slot[hi] = lo
__global__ __launch_bounds__(kBlock) void bucket_head_kernel(const int4* __restrict__ a, int64_t T, bool by_p,
                                                             int32_t* __restrict__ slot) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        const int4 t = a[i];
        const int32_t hi = by_p ? t.x : t.z;
        const int32_t lo = by_p ? t.y : t.x;
        bool head = i == 0;
        if (!head) {
            const int4 s = a[i - 1];
            head = (by_p ? s.x : s.z) != hi;
        }
        if (head) slot[hi] = lo;
    }
}

// last tuple of each bucket sorted by (r, p): slot[r] = the bucket's largest p
__global__ __launch_bounds__(kBlock) void bucket_tail_kernel(const int4* __restrict__ a, int64_t T,
                                                             int32_t* __restrict__ slot) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        const int4 t = a[i];
        const bool tail = i == T - 1 || a[i + 1].z != t.z;
        if (tail) slot[t.z] = t.x;
    }
}

// potentially completed: the bucket's largest p (slot2[r]) equals its
// smallest (q, just nominated); a tuple that is not clears its partition's
// flag in allpot (set to 1 for every vertex beforehand)
__global__ __launch_bounds__(kBlock) void potential_kernel(int4* __restrict__ a, int64_t T,
                                                           const int32_t* __restrict__ slot2,
                                                           uint32_t* __restrict__ allpot) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        const int4 t = a[i];
        const bool pot = slot2[t.z] == t.y;
        if (pot) a[i].w = t.w | kPot;
        else allpot[t.x] = 0u;
    }
}

// nominate: q <- slot[r] (u_min of the vertex bucket)
__global__ __launch_bounds__(kBlock) void nominate_kernel(int4* __restrict__ a, int64_t T,
                                                          const int32_t* __restrict__ slot) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) a[i].y = slot[a[i].z];
}

// join: p <- slot[p] (p_min of the partition bucket); *changed = 1 if any
// tuple moved.  mark (optional): mark[p_min] = 1 for the temporary tuples.
// allpot (optional, exclusion): a tuple whose partition did not move and whose
// partition's tuples are all potentially completed is done: labels[r] = p, it
// is flagged to leave the array, and it gets no temporary tuple.
__global__ __launch_bounds__(kBlock) void join_kernel(int4* __restrict__ a, int64_t T,
                                                      const int32_t* __restrict__ slot, uint32_t* __restrict__ mark,
                                                      const uint32_t* __restrict__ allpot,
                                                      int32_t* __restrict__ labels,
                                                      unsigned long long* __restrict__ changed) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    bool moved = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        const int4 t = a[i];
        const int32_t p = t.x;
        const int32_t pm = slot[p];
        moved |= pm != p;
        const bool done = allpot && pm == p && allpot[p] != 0u;
        a[i].x = pm;
        if (done) {
            a[i].w = t.w | kDone;
            labels[t.z] = p;
        } else if (mark) {
            mark[pm] = 1u;
        }
    }
    if (ballot(moved) && lane_id() == 0) atomic_add_agent(changed, 1ull);
}

__global__ __launch_bounds__(kBlock) void tuples_init_kernel(const int32_t* __restrict__ u,
                                                             const int32_t* __restrict__ v, int64_t m, int32_t n,
                                                             int4* __restrict__ a,
                                                             unsigned long long* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t T = (int64_t)n + 2 * m;
    uint32_t nbad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        if (i < n) {
            a[i] = make_int4((int32_t)i, kNone, (int32_t)i, 0);
        } else {
            const int64_t e = (i - n) >> 1;
            const int32_t x = u[e], y = v[e];
            const bool ok = (uint32_t)x < (uint32_t)n && (uint32_t)y < (uint32_t)n;
            nbad += ok ? 0u : 1u;
            const int32_t s = ok ? x : 0, d = ok ? y : 0;   // out-of-range: a harmless <0, _, 0>
            a[i] = ((i - n) & 1) ? make_int4(d, kNone, s, 0) : make_int4(s, kNone, d, 0);
        }
    }
    for (int off = 32; off > 0; off >>= 1) nbad += __shfl_xor(nbad, off);
    if (lane_id() == 0 && nbad) atomic_add_agent(bad, (unsigned long long)nbad);
}

__global__ __launch_bounds__(kBlock) void tuples_label_kernel(const int4* __restrict__ a, int64_t T,
                                                              int32_t* __restrict__ labels) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < T; i += stride) {
        const int4 t = a[i];
        labels[t.z] = t.x;   // every tuple of vertex r holds the same p at convergence
    }
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* __restrict__ x, int64_t n, uint32_t val) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = val;
}

static int grid_t(int64_t items) {
    int64_t g = (items + 4 * kBlock - 1) / (4 * kBlock);
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

// scan functors
struct DigitCount {
    const uint32_t* c;
    __device__ uint32_t operator()(int64_t i) const { return c[i]; }
};
struct DigitEmit {
    uint32_t* o;
    __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { o[i] = pre; }
};
struct MarkCount {
    const uint32_t* mark;
    __device__ uint32_t operator()(int64_t x) const { return mark[x]; }
};
struct TmpEmit {   // a temporary tuple <x, _, x> per marked x, after the T tuples
    int4* a;
    int64_t T;
    __device__ void operator()(int64_t x, uint32_t pre, uint32_t c) const {
        if (c) a[T + pre] = make_int4((int32_t)x, kNone, (int32_t)x, kTmp);
    }
};
struct KeepCount {   // tuples that are neither temporary nor done
    const int4* a;
    __device__ uint32_t operator()(int64_t i) const { return (a[i].w & (kTmp | kDone)) == 0 ? 1u : 0u; }
};
struct KeepEmit {   // kept tuples, their potential-completion flag cleared
    const int4* a;
    int4* out;
    __device__ void operator()(int64_t i, uint32_t pre, uint32_t c) const {
        if (c) {
            int4 t = a[i];
            t.w &= ~kPot;
            out[pre] = t;
        }
    }
};

struct TupleRun {
    hipStream_t s;
    int4* a;          // current array
    int4* b;          // other buffer
    uint32_t* counts; // 256 x tiles
    uint32_t* offs;
    uint32_t* bsum;
    unsigned long long* ctl;   // [0] changed, [1] changed (2nd join), [2] scan total, [3] range errors
    int32_t* slot;
    uint32_t* mark;
    int32_t n;
    int bits;
    int passes_per_sort;
    int64_t sorts = 0;
};

// stable sort of a[0..T) by (r, p) or (p, q); result in r.a
static hipError_t sort_tuples(TupleRun& r, int64_t T, bool by_p) {
    const int64_t nt = (T + kRsTile - 1) / kRsTile;
    if (nt > INT32_MAX) return hipErrorInvalidValue;
    for (int pass = 0; pass < r.passes_per_sort; ++pass) {
        const int shift = 8 * pass;
        rs_hist_kernel<<<(unsigned)nt, kRsThreads, 0, r.s>>>(r.a, T, by_p, r.bits, shift, nt, r.counts);
        hipError_t e = device_scan(DigitCount{r.counts}, DigitEmit{r.offs}, 256 * nt, r.bsum, r.ctl + 2, r.s);
        if (e != hipSuccess) return e;
        rs_scatter_kernel<<<(unsigned)nt, kRsThreads, 0, r.s>>>(r.a, r.b, T, by_p, r.bits, shift, nt, r.offs);
        std::swap(r.a, r.b);
    }
    ++r.sorts;
    return hipGetLastError();
}

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_label_tuples(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream,
                           int32_t exclude, cc_tuple_stats* st) {
    if (st) memset(st, 0, sizeof *st);
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size (m=%lld, n=%d)", (long long)m, n);
    if (m > 0 && n == 0) return fail(CC_EINVAL, "edges given for an empty vertex set");
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge array");
    if (n > 0 && !labels) return fail(CC_EINVAL, "NULL labels");
    const int64_t T0 = (int64_t)n + 2 * m;
    const int64_t cap = T0 + n;   // with one temporary tuple per partition at most
    if (cap >= ((int64_t)1 << 32)) return fail(CC_EINVAL, "too many tuples (n + 2m + n >= 2^32)");
    if (n == 0) return CC_OK;
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::unique_lock<std::mutex> lk(ws->mu);
    const int64_t ntmax = (cap + kRsTile - 1) / kRsTile;
    void *pa, *pb, *pc, *po, *ps, *pk, *pm, *pbs;
    const size_t tb = (size_t)cap * sizeof(int4);
    if ((rc = ws->get(WS_EDGES0, tb, &pa))) return rc;
    if ((rc = ws->get(WS_EDGES1, tb, &pb))) return rc;
    if ((rc = ws->get(WS_HIST, (size_t)256 * ntmax * sizeof(uint32_t), &pc))) return rc;
    if ((rc = ws->get(WS_OFF, (size_t)256 * ntmax * sizeof(uint32_t), &po))) return rc;
    if ((rc = ws->get(WS_SEGCOUNT, (size_t)scan_tiles(std::max<int64_t>(256 * ntmax, cap)) * sizeof(uint32_t), &pbs)))
        return rc;
    if ((rc = ws->get(WS_DEG, (size_t)n * sizeof(int32_t), &ps))) return rc;
    if ((rc = ws->get(WS_TAIL, (size_t)n * sizeof(uint32_t), &pm))) return rc;
    void *ps2, *pap;
    if ((rc = ws->get(WS_QUEUE, (size_t)n * sizeof(int32_t), &ps2))) return rc;
    if ((rc = ws->get(WS_BITS, (size_t)n * sizeof(uint32_t), &pap))) return rc;
    int32_t* slot2 = (int32_t*)ps2;      // largest p of each vertex bucket (exclusion)
    uint32_t* allpot = (uint32_t*)pap;   // per partition: all of its tuples potentially completed
    if ((rc = ws->get(WS_TOTALS, 64 * sizeof(unsigned long long), &pk))) return rc;
    unsigned long long* host;
    if ((rc = ws->pinned((void**)&host))) return rc;
    TupleRun r;
    r.s = s;
    r.a = (int4*)pa;
    r.b = (int4*)pb;
    r.counts = (uint32_t*)pc;
    r.offs = (uint32_t*)po;
    r.bsum = (uint32_t*)pbs;
    r.ctl = (unsigned long long*)pk;
    r.slot = (int32_t*)ps;
    r.mark = (uint32_t*)pm;
    r.n = n;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
    r.bits = bits;
    r.passes_per_sort = (2 * bits + 7) / 8;

    hipEvent_t ev[2];
    const bool timing = st != nullptr;
    if (timing) {
        (void)create_timing_event(&ev[0]);
        (void)create_timing_event(&ev[1]);
    }
    double ms_sort = 0.0;
    auto t_host = std::chrono::steady_clock::now();
    auto fail_ev = [&](int code) {
        if (timing) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
        }
        return code;
    };
    // a sort bracketed by events (its device time is added to ms_sort)
    auto timed_sort = [&](int64_t T, bool by_p) -> hipError_t {
        if (timing) (void)hipEventRecord(ev[0], s);
        hipError_t e = sort_tuples(r, T, by_p);
        if (timing && e == hipSuccess) {
            (void)hipEventRecord(ev[1], s);
            (void)hipEventSynchronize(ev[1]);
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[0], ev[1]);
            ms_sort += t;
        }
        return e;
    };
    hipError_t e = hipMemsetAsync(r.ctl, 0, 8 * sizeof(unsigned long long), s);
    if (e == hipSuccess) {
        tuples_init_kernel<<<grid_t(T0), kBlock, 0, s>>>(u, v, m, n, r.a, r.ctl + 3);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return fail_ev(hip_fail(e, "tuple init"));
    int64_t T = T0;
    int it = 0;
    for (;;) {
        if (++it > 100000) return fail_ev(fail(CC_EINTERNAL, "Algorithm 1 did not converge"));
        if ((e = hipMemsetAsync(r.ctl, 0, 2 * sizeof(unsigned long long), s)) != hipSuccess) break;
        // first pair of groupings: every partition joins its minimum neighbour
        if ((e = timed_sort(T, false)) != hipSuccess) break;
        bucket_head_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, false, r.slot);
        nominate_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, r.slot);
        if (exclude) {
            bucket_tail_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, slot2);
            fill_u32_kernel<<<grid_t(n), kBlock, 0, s>>>(allpot, n, 1u);
            potential_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, slot2, allpot);
        }
        if ((e = timed_sort(T, true)) != hipSuccess) break;
        bucket_head_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, true, r.slot);
        fill_u32_kernel<<<grid_t(n), kBlock, 0, s>>>(r.mark, n, 0u);
        join_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, r.slot, r.mark, exclude ? allpot : nullptr, labels, r.ctl);
        if (exclude) {
            // completed partitions leave the array
            if ((e = device_scan(KeepCount{r.a}, KeepEmit{r.a, r.b}, T, r.bsum, r.ctl + 2, s)) != hipSuccess) break;
            std::swap(r.a, r.b);
            if ((e = hipMemcpyAsync(host, r.ctl + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) !=
                hipSuccess)
                break;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
            T = (int64_t)host[0];
            if (T == 0) break;   // every partition completed: nothing moved, nothing left
        }
        // temporary tuples <p_min, _, p_min>, one per partition of the result
        if ((e = device_scan(MarkCount{r.mark}, TmpEmit{r.a, T}, n, r.bsum, r.ctl + 2, s)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(host, r.ctl + 2, sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess)
            break;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        const int64_t T2 = T + (int64_t)host[0];
        // second pair: pointer doubling through the temporary tuples
        if ((e = timed_sort(T2, false)) != hipSuccess) break;
        bucket_head_kernel<<<grid_t(T2), kBlock, 0, s>>>(r.a, T2, false, r.slot);
        nominate_kernel<<<grid_t(T2), kBlock, 0, s>>>(r.a, T2, r.slot);
        if ((e = timed_sort(T2, true)) != hipSuccess) break;
        bucket_head_kernel<<<grid_t(T2), kBlock, 0, s>>>(r.a, T2, true, r.slot);
        join_kernel<<<grid_t(T2), kBlock, 0, s>>>(r.a, T2, r.slot, nullptr, nullptr, nullptr, r.ctl + 1);
        // erase the temporary tuples
        if ((e = device_scan(KeepCount{r.a}, KeepEmit{r.a, r.b}, T2, r.bsum, r.ctl + 2, s)) != hipSuccess) break;
        std::swap(r.a, r.b);
        if ((e = hipMemcpyAsync(host, r.ctl, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s)) != hipSuccess)
            break;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        if (host[3]) return fail_ev(fail(CC_ERANGE, "%llu edge endpoints outside [0, n)", host[3]));
        if ((int64_t)host[2] != T) return fail_ev(fail(CC_EINTERNAL, "tuple count changed across an iteration"));
        if (!host[0] && !host[1]) break;
    }
    if (e == hipSuccess) {
        tuples_label_kernel<<<grid_t(T), kBlock, 0, s>>>(r.a, T, labels);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_ev(hip_fail(e, "tuple iteration"));
    const double ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host).count();
    if (st) {
        st->iterations = it;
        st->sorts = (int32_t)r.sorts;
        st->passes_per_sort = r.passes_per_sort;
        st->tuples = T0;
        st->ms_sort = ms_sort;
        st->ms_total = ms_total;
    }
    return fail_ev(CC_OK);
}
