// Degree / histogram / CSR launch interface (degree.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmi {

constexpr int kBucketShift = 15;      // 32768 vertices per bucket (LDS counters)
constexpr int kMaxBuckets = 16384;    // n <= 2^29 for the bucketed degree pass
constexpr int kExactBins = 4096;      // exact degree histogram below this
constexpr int kBlockD = 1024;         // threads of the per-bucket kernel
constexpr int kStagedMaxB = 2048;     // one-level scatter up to this many buckets (n <= 2^26), else two levels
constexpr int kGrpShift = 8;          // CSR fill: vertices per group = 2^kGrpShift
constexpr int kGroups = 1 << (kBucketShift - kGrpShift);   // groups per bucket

struct BucketPlan {
    int32_t B;       // vertex buckets
    int32_t nblk;    // edge-chunk blocks
    int64_t chunk;   // edges per block
};

struct BucketBufs {
    uint32_t* counts;            // [B][nblk]: per-block counts, then their prefix over the blocks
    unsigned long long* tot;     // [B]
    unsigned long long* base;    // [B + 1]
    uint16_t* loc;               // [2m] endpoint id within its bucket, grouped by bucket
    int32_t* other;              // [2m] the other endpoint (CSR builds)
    uint32_t* loc32;             // [2m] first level when B > kStagedMaxB: id within the super-bucket
    int32_t* other32;            // [2m] its other ends (CSR builds)
    uint16_t* tloc;              // [2m] CSR fill: entries regrouped by 256-vertex group
    int32_t* tother;             // [2m]
    unsigned long long* err;     // range errors
    uint32_t* gcnt;              // [B * kGroups] CSR fill: entries of each group placed so far
    int64_t loc_cap = 0;         // 16-bit entries loc can hold (the capped layout needs more than 2m)
    int32_t capped_grid = 0;     // scatter blocks of a capped layout in counts (0: none)
    bool other_written = false;
    bool counted = false;        // counts / tot / base hold the counted layout's prefixes
};

// returns -1 if n is too large for the bucketed pass or m >= 2^31 (the
// per-bucket prefixes and the scatter's output slots are 32-bit)
int bucket_plan(int32_t n, int64_t m, BucketPlan* p);

// deg[n] (+ histograms when want_hist, + CSR off[n+1]/adj[2m] when want_csr).
// hist64/histx/tail_count/argmax_key must be zeroed by the caller.
// Degrees-only passes (want_csr = 0, allow_capped) may skip the count pass:
// small lists are counted straight from the edges in one launch, larger ones
// take the capped layout; err[1] (err must hold two words, both zeroed) then
// reports whether a run overflowed its capacity, in which case the results
// are void and the pass must be run again with allow_capped off.
hipError_t launch_bucket_degree(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                BucketBufs& w, int32_t* deg, int want_hist, unsigned long long* hist64,
                                unsigned long long* histx, int32_t* tail, int64_t tail_cap,
                                unsigned long long* tail_count, unsigned long long* argmax_key, int want_csr,
                                int64_t* off, int32_t* adj, hipStream_t s, bool allow_capped = false);

// CSR from an earlier launch_bucket_degree's buckets and deg[] (no recount);
// scatters the other endpoints first if that pass did not
hipError_t launch_bucket_csr_from_deg(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                      BucketBufs& w, int32_t* deg, int64_t* off, int32_t* adj, hipStream_t s);

hipError_t launch_degree_hist(const int32_t* deg, int32_t n, unsigned long long* hist64, unsigned long long* histx,
                              int32_t* tail, int64_t tail_cap, unsigned long long* tail_count,
                              unsigned long long* argmax_key, hipStream_t s);

}  // namespace ccmi
