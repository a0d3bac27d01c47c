// Device-wide exclusive scan of 32-bit counts given by a functor, in three
// launches: per-block totals, one workgroup scanning the block totals, and a
// second pass that rescans each block with its offset and hands every item
// its exclusive prefix.  Used for compactions (the 64-bit relabel's slot
// numbering, the tuple array's temporary tuples).
#pragma once

#include "common.hpp"

namespace ccmi {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;                                 // items per thread
constexpr int64_t kScanTile = (int64_t)kScanThreads * kScanPer;

// inclusive scan of v over the workgroup; *total gets the workgroup sum
__device__ __forceinline__ uint32_t scan_block_incl(uint32_t v, uint32_t* lds_w, uint32_t* total) {
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_w[w] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int nw = kScanThreads / 64;
        uint32_t s = threadIdx.x < nw ? lds_w[threadIdx.x] : 0u;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(s, off);
            if (lane >= off) s += y;
        }
        if (threadIdx.x < nw) lds_w[threadIdx.x] = s;   // inclusive over waves
    }
    __syncthreads();
    const uint32_t before = w > 0 ? lds_w[w - 1] : 0u;
    *total = lds_w[kScanThreads / 64 - 1];
    __syncthreads();
    return before + x;
}

// phase 1: bsum[b] = sum of count(i) over tile b
template <class Count>
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(Count count, int64_t n, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t lds_w[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) s += count(base + k);
    uint32_t tot;
    (void)scan_block_incl(s, lds_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// phase 2 (one workgroup): bsum[0..nb) -> exclusive prefixes; *total = sum
static __global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint32_t* __restrict__ bsum, int64_t nb,
                                                                 unsigned long long* __restrict__ total) {
    __shared__ uint32_t lds_w[kScanThreads / 64];
    const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t lo = (int64_t)threadIdx.x * per;
    const int64_t hi = lo + per < nb ? lo + per : nb;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += bsum[i];
    uint32_t tot;
    uint32_t run = scan_block_incl(s, lds_w, &tot) - s;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = bsum[i];
        bsum[i] = run;
        run += c;
    }
    if (threadIdx.x == 0) *total = tot;
}

// phase 3: emit(i, exclusive prefix of item i, count(i)) for every item
template <class Count, class Emit>
__global__ __launch_bounds__(kScanThreads) void scan_emit_kernel(Count count, Emit emit, int64_t n,
                                                                 const uint32_t* __restrict__ boff) {
    __shared__ uint32_t lds_w[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    uint32_t c[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = base + k < n ? count(base + k) : 0u;
        s += c[k];
    }
    uint32_t tot;
    uint32_t run = boff[blockIdx.x] + scan_block_incl(s, lds_w, &tot) - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) emit(base + k, run, c[k]);
        run += c[k];
    }
}

inline int64_t scan_tiles(int64_t n) { return n > 0 ? (n + kScanTile - 1) / kScanTile : 1; }

// Runs the three phases on stream s.  bsum: scan_tiles(n) words of scratch;
// total: one device word, the sum of all counts (it must stay below 2^32).
template <class Count, class Emit>
hipError_t device_scan(Count count, Emit emit, int64_t n, uint32_t* bsum, unsigned long long* total, hipStream_t s) {
    const int64_t nb = scan_tiles(n);
    if (nb > INT32_MAX) return hipErrorInvalidValue;
    scan_tiles_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(count, n, bsum);
    scan_sums_kernel<<<1, kScanThreads, 0, s>>>(bsum, nb, total);
    scan_emit_kernel<<<(unsigned)nb, kScanThreads, 0, s>>>(count, emit, n, bsum);
    return hipGetLastError();
}

}  // namespace ccmi
