// Device body of one SV pass over a block's edge segment (hook + compact),
// shared by the single-graph passes (sv.hip) and the persistent batched
// kernel (batched.hip).
#pragma once

#include "common.hpp"

namespace ccmi {

constexpr int kEPT = 4;   // edges per thread per tile

// Process `len` edges of this block.  loader(t0, a, c, valid) fills this
// thread's kEPT edges of the tile that starts at edge t0 of the segment
// (edge t0 + threadIdx.x + k * kBlock in slot k; valid[k] false for an edge
// past the end or one to skip).  A loader that issues all of its reads
// before it uses any lets them overlap: each edge's reads then cost one
// memory round trip per tile instead of one per edge.
//
// Per edge: find both roots; if they differ, hook the larger root below the
// smaller with atomicMin.  The edge is finished (dropped) when its roots
// agree or when its hook lands on a root (the two trees are then one).  If
// the atomic finds hi already linked to old != hi, the pair still to be
// joined is (old, lo) -- hi ~ lo is now a link when old > lo, hi ~ old when
// old < lo -- and up to max_link attempts are made in this pass; an edge not
// finished by then is kept as that pair.  max_link = 1 is the plain SV pass
// (one hook per edge per pass, the rest waits for the next pass).
//
// A find stops after kMaxHops links.  An edge whose find stopped short of a
// root is kept as the pair of vertices reached (each is an ancestor of its
// endpoint, so the pair carries the edge's connection) and counted in nlong
// (per thread); its caller then flattens the forest before the next pass.
//
// Survivors go to dst[kept_off ...] (if write_out), roots hooked in this pass
// to hdst[hook_off ...].  Offsets are block-uniform running counts.
//
// Per thread, natom counts the atomics issued and nchase the parent[] reads
// beyond the two first-level gathers per edge (the walks up the forest), for
// the byte model; callers that do not report them let the compiler drop them.
template <class Loader>
__device__ __forceinline__ void sv_segment(int64_t len, Loader loader, int32_t* parent, int2* __restrict__ dst,
                                           int32_t* __restrict__ hdst, bool write_out, int max_link,
                                           uint32_t& kept_off, uint32_t& hook_off, uint32_t& nlong,
                                           uint32_t* lds, uint32_t& natom, uint32_t& nchase) {
    for (int64_t t0 = 0; t0 < len; t0 += kBlock * kEPT) {
        int32_t a[kEPT], c[kEPT], pa[kEPT], pc[kEPT];
        bool valid[kEPT];
        loader(t0, a, c, valid);
        // all first-level gathers before any dependent chase
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            if (valid[k]) {
                pa[k] = parent[a[k]];
                pc[k] = parent[c[k]];
            }
        }
        // Walk the 2 * kEPT root chains of this thread in lockstep: every
        // step issues the next load of each unfinished chain before using
        // any, so the dependent loads of different chains overlap instead of
        // queueing behind each other.  a[k] / c[k] become the roots; after
        // kMaxHops steps (cut) a chain still moving stops where it is, and
        // is recognised below by pa[k] != a[k] (or pc[k] != c[k]).
        bool cut = false;
        for (int hop = 0;; ++hop) {
            bool more = false, mva[kEPT], mvc[kEPT];
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                mva[k] = valid[k] && pa[k] != a[k];
                mvc[k] = valid[k] && pc[k] != c[k];
                more |= mva[k] | mvc[k];
            }
            if (!more) break;
            if (hop == kMaxHops) {
                cut = true;
                break;
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                if (mva[k]) a[k] = pa[k];
                if (mvc[k]) c[k] = pc[k];
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                if (mva[k]) pa[k] = parent[a[k]];
                if (mvc[k]) pc[k] = parent[c[k]];
                nchase += (uint32_t)mva[k] + (uint32_t)mvc[k];
            }
        }
        bool keep[kEPT], hk[kEPT], go[kEPT];
        int2 e[kEPT];
        int32_t hroot[kEPT], lo[kEPT], hi[kEPT], old[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            keep[k] = false;
            hk[k] = false;
            go[k] = false;
            hroot[k] = 0;
            lo[k] = hi[k] = 0;
            if (!valid[k]) continue;
            const int32_t ra = a[k];
            const int32_t rc = c[k];
            if (cut && (pa[k] != ra || pc[k] != rc)) {   // a find stopped short of a root
                ++nlong;
                if (ra != rc) {
                    keep[k] = true;
                    e[k] = make_int2(ra, rc);
                }
                continue;
            }
            go[k] = ra != rc;
            lo[k] = ra < rc ? ra : rc;
            hi[k] = ra < rc ? rc : ra;
        }
        // first hook attempt of every edge of the thread, all in flight together
#pragma unroll
        for (int k = 0; k < kEPT; ++k)
            if (go[k]) {
                old[k] = atomic_min_agent(&parent[hi[k]], lo[k]);   // hook the larger root
                ++natom;
            }
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            if (!go[k]) continue;
            int32_t o = old[k], l = lo[k], h = hi[k];
            for (int tries = 1;;) {
                if (o == h) {              // h was a root: the two trees are joined
                    hk[k] = true;
                    hroot[k] = h;
                    break;
                }
                if (tries >= max_link) {
                    keep[k] = true;
                    e[k] = o > l ? make_int2(o, h) : make_int2(l, h);
                    break;
                }
                bool root_a, root_c;
                const int32_t ra = find_bounded(parent, o, &root_a);
                const int32_t rc = find_bounded(parent, l, &root_c);
                nchase += 2;   // at least one read each (deeper walks are not counted)
                if (!(root_a && root_c)) {   // keep the pair still to be joined, as ancestors
                    ++nlong;
                    if (ra != rc) {
                        keep[k] = true;
                        e[k] = make_int2(ra, rc);
                    }
                    break;
                }
                if (ra == rc) break;       // joined meanwhile: finished
                l = ra < rc ? ra : rc;
                h = ra < rc ? rc : ra;
                o = atomic_min_agent(&parent[h], l);
                ++natom;
                ++tries;
            }
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
            if (hk[k]) hdst[hoff + hpre[k]] = hroot[k];
        }
        kept_off += tot & 0xffffu;
        hook_off += tot >> 16;
    }
}

}  // namespace ccmi
