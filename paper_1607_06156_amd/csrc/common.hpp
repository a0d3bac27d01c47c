// Shared device helpers and internal launch interfaces of libccmi (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmi {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;

// -------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of mask in lanes below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// agent-scope atomics (coherent across the XCDs of one device)
__device__ __forceinline__ int32_t atomic_min_agent(int32_t* p, int32_t v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t atomic_add_agent(unsigned long long* p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_or_agent(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Longest walk up the parent forest taken in one go.  Trees are shallow on
// the workloads of Section V, but one pass can link a long run of vertices
// at once (a path whose ids and edge order both follow it hooks every vertex
// onto its predecessor concurrently), and an unbounded walk from each vertex
// of such a chain costs time quadratic in its length.  A walk that reaches
// this bound stops at the ancestor it reached; the flatten rounds (each
// moves every vertex at least this far up) finish the chain.
constexpr int kMaxHops = 64;

// Walk from x towards its root, at most kMaxHops links; returns the vertex
// reached and sets *root when it is a root.  parent[] may change concurrently
// (hooks by other lanes) and a plain load may return an older value, but
// every value parent[x] ever holds is an id <= x of a vertex connected to x,
// so the walk strictly descends and ends at an ancestor of x (a root when
// *root, as it was when read).
__device__ __forceinline__ int32_t find_bounded(const int32_t* parent, int32_t x, bool* root) {
    int32_t p = parent[x];
    for (int h = 0; h < kMaxHops && p != x; ++h) {
        x = p;
        p = parent[x];
    }
    *root = p == x;
    return x;
}

// Block-wide exclusive prefix of per-wave totals; returns this wave's offset
// within the block and writes the block total to *total.  lds must hold
// kWaves + 1 uint32.
__device__ __forceinline__ uint32_t block_wave_offset(uint32_t wave_total, uint32_t* lds, uint32_t* total) {
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0) lds[wave] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < kWaves; ++w) { uint32_t t = lds[w]; lds[w] = acc; acc += t; }
        lds[kWaves] = acc;
    }
    __syncthreads();
    uint32_t off = lds[wave];
    *total = lds[kWaves];
    __syncthreads();
    return off;
}

// ------------------------------------------------------ segmented edge lists
// Active edges live in per-block segments: block b of a pass owns slots
// [b * cap, b * cap + count[b]) of an int2 buffer (x = smaller root, y =
// larger).  Passes keep the block count fixed, so block b reads its own
// segment and writes its survivors to the same slots of the other buffer;
// no global atomic is needed to place output.
struct SegList {
    int2* buf;
    int64_t cap;        // slots per segment
    int32_t nseg;       // segments (= blocks)
    uint32_t* count;    // device, nseg entries
};

// ------------------------------------------------------ launch interfaces
// All launchers enqueue on `s` and return the hipError_t of the launch.

// SV (sv.hip)
hipError_t launch_sv_init(int32_t* parent, int32_t n, hipStream_t s);
// first pass over the caller's SoA edge list (dense, m edges), cut into
// out.nseg segments of out.cap edges; this launch covers segments
// [seg0, seg0 + nblocks), one block each.  Writes survivors into out (if
// write_out), hooked roots into hooked (segments of the same cap), per-segment
// counts, per-segment statistics (segstat[3 b ...]: atomics issued, chase
// reads, edges dropped by the bitmap), and accumulates totals[2] (range
// errors) and totals[4] (edges whose find stopped at the hop bound: the
// forest needs flatten rounds).  With gbits and gflag (from launch_giant_pick
// and launch_giant_bits after a flatten), edges with both endpoints in the
// largest tree are dropped on a bitmap probe.
hipError_t launch_sv_pass_soa(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* parent,
                              SegList out, int32_t seg0, int32_t nblocks, int write_out, int max_link,
                              int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                              uint32_t* segstat, const uint32_t* gbits, const int32_t* gflag, hipStream_t s);
// passes over a segmented list: segments [seg0, seg0 + nblocks) of in, each
// one block, survivors to the same segments of out
hipError_t launch_sv_pass_seg(SegList in, int32_t seg0, int32_t nblocks, int32_t* parent, SegList out, int write_out,
                              int max_link, int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                              uint32_t* segstat, hipStream_t s);
// largest tree of a flattened forest, by sampling: *gflag = its root, or -1
// if no root holds 1/16 of the samples.  No hook may run concurrently.
hipError_t launch_giant_pick(const int32_t* parent, int32_t n, int32_t* gflag, hipStream_t s);
// bits (2 * ceil(n / 64) words) = membership of the tree of *gflag (if >= 0),
// right after a flatten.  No hook may run concurrently.
hipError_t launch_giant_bits(const int32_t* parent, int32_t n, const int32_t* gflag, uint32_t* bits, hipStream_t s);
// pointer-jumps the hooked roots of each segment, at most kMaxHops links each
// (no hook may run concurrently)
hipError_t launch_sv_shortcut(int32_t* parent, const int32_t* hooked, const uint32_t* hooked_count, int64_t cap,
                              int32_t nseg, hipStream_t s);
// totals[0] = sum(kept_count), totals[1] = sum(hooked_count) over nseg
// segments, totals[3] = sum(hooked_count) over segments seg_lo .. nseg-1,
// totals[7..9] = sums of the segments' statistics
hipError_t launch_sv_totals(const uint32_t* hooked_count, const uint32_t* kept_count, int32_t nseg, int32_t seg_lo,
                            const uint32_t* segstat, unsigned long long* totals, hipStream_t s);
// one flatten round: parent[x] = root(x) for every x whose root lies at most
// kMaxHops links up, else the ancestor that far up, and then *open = 1 (set
// only, never cleared here).  No hook may run concurrently.
hipError_t launch_sv_finalize(int32_t* parent, int32_t n, unsigned long long* open, hipStream_t s);

}  // namespace ccmi
