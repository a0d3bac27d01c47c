// Batched-mode launch interface (batched.hip, batched_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmi {

struct BatchArgsHost {
    const int32_t* u;
    const int32_t* v;
    const int64_t* edge_off;
    const int64_t* vert_off;
    int32_t G;
    int64_t m;
    int32_t n;
    int32_t* labels;
    int2* buf0;
    int2* buf1;
    unsigned long long* part;   // 6 x blocks partials (survivors, hooks, bounded finds; 2 arrays each)
    unsigned long long* bstat;  // 4 x blocks: atomics, walk reads, edges read, survivors written
    uint32_t* cnt0;
    uint32_t* cnt1;
    uint32_t* hcnt;
    int32_t* hooked;
    unsigned int* bar;
    unsigned long long* status;
    int32_t max_passes;
    int32_t max_link;
    uint64_t barrier_ticks;     // grid-barrier spin limit (100 MHz wall-clock ticks)
};

constexpr int64_t kBatchTile = 1024;   // edges per tile (256 threads x 4)

// largest co-resident grid of the persistent kernel on the current device
hipError_t batched_max_blocks(int* blocks);
// one cooperative launch running the whole SV loop over all graphs
hipError_t launch_batched(const BatchArgsHost& h, int blocks, hipStream_t s);

// fallback without a persistent grid: the batch as one disjoint-union graph
// (global ids; -1 for an id outside its graph; *bad counts decreasing offsets)
hipError_t launch_union_relabel(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                                int32_t G, int64_t m, int32_t* gu, int32_t* gv, unsigned long long* bad,
                                hipStream_t s);
// labels[x] -= vert_off[graph of x]
hipError_t launch_union_unshift(int32_t* labels, const int64_t* vert_off, int32_t G, int64_t n, hipStream_t s);

}  // namespace ccmi
