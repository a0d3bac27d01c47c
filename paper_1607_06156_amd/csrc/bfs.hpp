// BFS / filter launch interface (bfs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace ccmi {

constexpr double kBeamerAlpha = 14.0;
constexpr double kBeamerBeta = 24.0;

// pre[0..qn] = exclusive prefix of frontier degrees; bsum needs ceil(qn/1024) entries
hipError_t launch_qdeg_scan(const int32_t* q, int64_t qn, const int64_t* off, int64_t* pre, int64_t* bsum,
                            int64_t* total, hipStream_t s);
// ctr[0] += new vertices (appended to nq), ctr[1] += their degrees
hipError_t launch_topdown(const int32_t* q, int64_t qn, const int64_t* pre, int64_t total_entries,
                          const int64_t* off, const int32_t* adj, uint32_t* vis, int32_t* nq,
                          unsigned long long* ctr, hipStream_t s);
// ctr[0] += new vertices (bits in next), ctr[1] += their degrees, ctr[2] += entries examined
hipError_t launch_bottomup(int32_t n, const int64_t* off, const int32_t* adj, uint32_t* vis, const uint32_t* front,
                           uint32_t* next, unsigned long long* ctr, hipStream_t s);
// Consecutive top-down levels in one workgroup, from the frontier in qa (qn
// vertices, already marked in vis), while a level's frontier has at most
// max_entries adjacency entries and for at most max_levels levels; the
// frontier it stops at is left in qa.  qa / qb hold n entries, pre n + 1.
// out[0..6): levels, vertices visited, entries examined, degree sum of the
// vertices visited, frontier size left, its degree sum.
constexpr int64_t kFewLevelEntries = 65536;   // largest frontier (in entries) it expands
hipError_t launch_bfs_few(const int64_t* off, const int32_t* adj, int32_t* qa, int32_t* qb, int64_t qn,
                          int64_t max_entries, int32_t max_levels, uint32_t* vis, int64_t* pre,
                          unsigned long long* out, hipStream_t s);
hipError_t launch_queue_to_bits(const int32_t* q, int64_t qn, uint32_t* bits, hipStream_t s);
hipError_t launch_bits_to_queue(const uint32_t* bits, int64_t words, int32_t* q, unsigned long long* qn,
                                hipStream_t s);
// *label (pre-set to INT32_MAX) = min visited id; labels[x] = visited ? *label : x
hipError_t launch_bfs_label(const uint32_t* vis, int32_t n, int32_t* label, int32_t* labels, hipStream_t s);
// edges whose first endpoint is unvisited -> segments of out; *total = their count
// (*bad += edges with an endpoint outside [0, n); those are dropped)
hipError_t launch_filter(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const uint32_t* vis, SegList out,
                         unsigned long long* total, unsigned long long* bad, hipStream_t s);
// *bad += violations of the CSR contract (offsets, entry range)
// The edges between unvisited vertices from the CSR rows of the unvisited
// vertices, as (smaller, larger) pairs (a self-loop once per two entries).
// Count: per-wave counts into wcount[rest_waves(n)], turned into an exclusive
// prefix in place, *total = their sum.  Emit: the edges into fu, fv (room for
// *total each) at those offsets.
int64_t rest_waves(int32_t n);
hipError_t launch_rest_count(const uint32_t* vis, const int64_t* off, const int32_t* adj, int32_t n, int64_t* wcount,
                             int64_t* total, hipStream_t s);
hipError_t launch_rest_emit(const uint32_t* vis, const int64_t* off, const int32_t* adj, int32_t n,
                            const int64_t* woff, int32_t* fu, int32_t* fv, hipStream_t s);
hipError_t launch_csr_check(const int64_t* off, int32_t n, const int32_t* adj, int64_t nadj,
                            unsigned long long* bad, hipStream_t s);
hipError_t launch_seg_to_soa(SegList in, int64_t* prefix_scratch, int64_t* total_scratch, int32_t* fu, int32_t* fv,
                             hipStream_t s);

}  // namespace ccmi
