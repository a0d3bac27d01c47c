// Hubs of a power-law graph during the first SV pass.
//
// On a power-law graph a few vertices of the highest degree hold a large share
// of the edge endpoints (R-MAT scale 24, edge factor 16: the 2048 largest hold
// 12.6 % of them).  When the degrees are known (the heuristic route computes
// them for the power-law fit of Section IV), the filtered launches of the
// first pass answer the largest-tree probes of those vertices from a table in
// LDS instead of the bitmap in L2.  The table is an exact subset of the
// bitmap: a hub is listed iff its bit is set.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ccmi {

constexpr int kHubMax = 2048;             // hubs listed at most
constexpr int kHubBits = 10;
constexpr int kHubBuckets = 1 << kHubBits;   // table buckets of 4 vertex ids (16 KB)
constexpr int64_t kHubMinDegree = 256;    // no vertex of smaller degree is a hub

// Bytes of the hub arrays: the list (kHubMax ids), the table of every listed
// hub and the table of those in the largest tree.
constexpr size_t kHubBytes = (size_t)kHubMax * 4 + (size_t)kHubBuckets * 16 * 2;

// The vertices x with deg[x] >= dmin, at most kHubMax of them (dmin is chosen
// so that no more exist): their ids in list[], how many in *count (which the
// caller zeroes first), and a table of them in ids[] (kHubBuckets int4 of
// vertex ids, -1 in empty slots; a hub whose bucket is full is left out).
hipError_t launch_hub_list(const int32_t* deg, int32_t n, int32_t dmin, int32_t* list, uint32_t* count, int4* ids,
                           hipStream_t s);

// launch_giant_bits that also writes tree_ids: ids[] with every hub outside
// the tree of *gflag replaced by -1 (nothing when *gflag is -1).
hipError_t launch_giant_bits_hubs(const int32_t* parent, int32_t n, const int32_t* gflag, uint32_t* bits,
                                  const int4* ids, int4* tree_ids, hipStream_t s);

// launch_sv_pass_soa whose filtered launch (gbits and gflag given) also
// takes tree_ids (from launch_giant_bits_hubs after the same pick): the
// probes of the hubs it lists are answered from LDS.
hipError_t launch_sv_pass_soa_hubs(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* parent,
                                   SegList out, int32_t seg0, int32_t nblocks, int write_out, int max_link,
                                   int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                                   uint32_t* segstat, const uint32_t* gbits, const int32_t* gflag,
                                   const int4* tree_ids, hipStream_t s);

}  // namespace ccmi
