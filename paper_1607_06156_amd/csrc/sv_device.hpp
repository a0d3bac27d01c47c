// Device body of one SV pass over a block's edge segment (hook + compact),
// shared by the single-graph passes (sv.hip) and the persistent batched
// kernel (batched.hip).
#pragma once

#include "common.hpp"

namespace ccmi {

constexpr int kEPT = 4;   // edges per thread per tile

// Process `len` edges of this block.  load(i, &a, &c) fetches edge i of the
// segment as two vertex ids and returns false to skip it.  Survivors go to
// dst[kept_off ...] (if write_out), roots hooked for the first time in this
// pass to hdst[hook_off ...].  Offsets are block-uniform running counts.
template <class Load>
__device__ __forceinline__ void sv_segment(int64_t len, Load load, int32_t* parent, int2* __restrict__ dst,
                                           int32_t* __restrict__ hdst, bool write_out, uint32_t& kept_off,
                                           uint32_t& hook_off, uint32_t* lds) {
    for (int64_t t0 = 0; t0 < len; t0 += kBlock * kEPT) {
        int32_t a[kEPT], c[kEPT], pa[kEPT], pc[kEPT];
        bool valid[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            const int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
            valid[k] = i < len && load(i, &a[k], &c[k]);
        }
        // all first-level gathers before any dependent chase
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            if (valid[k]) {
                pa[k] = parent[a[k]];
                pc[k] = parent[c[k]];
            }
        }
        bool keep[kEPT], hk[kEPT];
        int2 e[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            keep[k] = false;
            hk[k] = false;
            if (!valid[k]) continue;
            const int32_t ra = pa[k] == a[k] ? a[k] : find_root(parent, pa[k]);
            const int32_t rc = pc[k] == c[k] ? c[k] : find_root(parent, pc[k]);
            if (ra == rc) continue;                       // finished: both ends share a root
            const int32_t lo = ra < rc ? ra : rc;
            const int32_t hi = ra < rc ? rc : ra;
            const int32_t old = atomic_min_agent(&parent[hi], lo);   // hook the larger root
            hk[k] = (old == hi);
            keep[k] = true;
            // If hi had already been linked to some lo < old < hi, the atomic replaced
            // that link: carry the displaced connection (old, hi) instead (hi ~ lo is now
            // a forest link).  Connectivity of forest + active edges is then preserved
            // whatever parent[] values the finds read.
            e[k] = (old != hi && old > lo) ? make_int2(old, hi) : make_int2(lo, hi);
        }
        // wave ballots -> slot prefixes; one block scan of packed (kept | hooks << 16)
        uint64_t km[kEPT], hm[kEPT];
        uint32_t kpre[kEPT], hpre[kEPT];
        uint32_t wk = 0, wh = 0;
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            km[k] = ballot(keep[k]);
            hm[k] = ballot(hk[k]);
            kpre[k] = wk + lanes_below(km[k]);
            hpre[k] = wh + lanes_below(hm[k]);
            wk += (uint32_t)__popcll(km[k]);
            wh += (uint32_t)__popcll(hm[k]);
        }
        uint32_t tot;
        const uint32_t woff = block_wave_offset(wk | (wh << 16), lds, &tot);
        const uint32_t koff = kept_off + (woff & 0xffffu), hoff = hook_off + (woff >> 16);
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            if (write_out && keep[k]) dst[koff + kpre[k]] = e[k];
            if (hk[k]) hdst[hoff + hpre[k]] = e[k].y;
        }
        kept_off += tot & 0xffffu;
        hook_off += tot >> 16;
    }
}

}  // namespace ccmi
