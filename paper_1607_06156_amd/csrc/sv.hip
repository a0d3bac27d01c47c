// Shiloach-Vishkin style iteration on an edge list (Section III-A).
//
// The paper keeps tuples <p, q, r> and, per iteration, lets every partition p
// join its minimum neighbouring partition (two sorts), then pointer-jumps the
// joined partition once more (two more sorts), and drops completed partitions
// from the working set (Section III-A.4).  On one GPU the partition of vertex
// x is represented directly by a parent forest parent[] (labels_out doubles as
// parent), in which every root is the smallest id of its tree:
//
//  * hook    -- for each active edge with roots ra != rb, atomicMin(parent[max],
//               min): a partition joins the smallest neighbouring partition
//               that reaches it in this pass (the atomic keeps the minimum of
//               all candidates, as p_min = min C(p) does);
//  * shortcut-- each root hooked in the pass is pointed straight at its new
//               root (pointer jumping, Fig. "doubling"); every walk up the
//               forest stops after kMaxHops links, and flatten rounds finish
//               a deeper chain;
//  * compact -- an edge whose endpoints already share a root is finished and
//               dropped; survivors are rewritten as (root, root), so the next
//               pass starts from roots.  This is the exclusion of completed
//               work (Section III-A.4), applied per edge instead of per
//               partition.
//
// Invariant: parent[x] <= x, links only point to connected vertices, and the
// connectivity of (forest links + active edges) always equals that of the
// input.  Every change of parent[] by a hook is an atomicMin; when it replaces
// an existing link hi -> old by hi -> lo, the displaced pair (old, hi) stays
// active, so no connection is lost even if a find read an outdated parent.
// The loop ends when no edge is active, and the forest roots are then the
// component minima.
#include "common.hpp"
#include "hubs.hpp"
#include "sv_device.hpp"

namespace ccmi {

__global__ __launch_bounds__(kBlock) void sv_init_kernel(int32_t* __restrict__ parent, int32_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) parent[i] = (int32_t)i;
}

// Hub tables: kHubBuckets buckets of 4 vertex ids (-1 = empty), bucket by a
// multiplicative hash of the id.  A filtered launch of the first pass keeps
// the table of the largest tree's hubs in LDS and answers their probes there;
// an id that is not in it (its bucket was full, or it is no hub or not in the
// tree) is probed in the bitmap as before.
__device__ __forceinline__ uint32_t hub_bucket(int32_t x) { return ((uint32_t)x * 2654435761u) >> (32 - kHubBits); }

__device__ __forceinline__ bool in_hubs(const int4* lhub, int32_t x) {
    const int4 q = lhub[hub_bucket(x)];
    return (q.x == x) | (q.y == x) | (q.z == x) | (q.w == x);
}

// One pass: hook + compact over one block segment of edges.
// SOA: edges come from the caller's u[], v[] (dense); the block works on
// segment b = seg0 + blockIdx.x, edges [b*cap, min((b+1)*cap, m)), and checks
// ids against [0, n).  Else from segment b of `in`.
// FILT (SOA only): while *gflag >= 0, an edge whose two endpoints both have
// their bit set in gbits (vertices already in the largest tree when the
// bitmap was built) is finished and dropped without touching parent[].
// With hubt (FILT), the hubs that table lists take their bit from LDS.
// segstat[3 b ...] receives the block's atomics issued, chase reads and edges
// dropped by the bitmap.
template <bool SOA, bool FILT>
__global__ __launch_bounds__(kBlock) void sv_pass_kernel(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                                         int64_t m, int32_t n, int32_t seg0, SegList in,
                                                         int32_t* parent, SegList out, int write_out, int max_link,
                                                         int32_t* __restrict__ hooked,
                                                         uint32_t* __restrict__ hooked_count,
                                                         unsigned long long* __restrict__ totals,
                                                         const uint32_t* __restrict__ gbits,
                                                         const int32_t* __restrict__ gflag,
                                                         uint32_t* __restrict__ segstat,
                                                         const int4* __restrict__ hubt) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint32_t red[3][kWaves];
    __shared__ int4 lhub[FILT ? kHubBuckets : 1];   // the largest tree's hubs (filtered launches)
    const int b = seg0 + blockIdx.x;
    int2* dst = out.buf + (int64_t)b * out.cap;
    int32_t* hdst = hooked + (int64_t)b * out.cap;
    uint32_t kept_off = 0, hook_off = 0, bad = 0, nlong = 0, natom = 0, nchase = 0, nfilt = 0;
    if (SOA) {
        const int64_t base = (int64_t)b * out.cap;
        int64_t len = m - base;
        if (len > out.cap) len = out.cap;
        if (len < 0) len = 0;
        const bool filt = FILT && *gflag >= 0;
        // hubs of the largest tree: their probes are answered from LDS
        const bool hubs = filt && hubt != nullptr;
        if (FILT) {
            if (hubs)
                for (int i = threadIdx.x; i < kHubBuckets; i += kBlock) lhub[i] = hubt[i];
            __syncthreads();
        }
        // Every read of a tile goes out before any is used: the edges (read
        // once, with non-temporal loads that keep them from displacing
        // parent[] and the bitmap in the caches), then the bit probes.
        // Indices past the end read edge 0 of the segment and are dropped.
        auto loader = [&](int64_t t0, int32_t* a, int32_t* c, bool* valid) {
            int64_t idx[kEPT];
            bool in[kEPT];
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                const int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
                in[k] = i < len;
                idx[k] = base + (in[k] ? i : 0);
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                a[k] = __builtin_nontemporal_load(u + idx[k]);
                c[k] = __builtin_nontemporal_load(v + idx[k]);
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                const bool ok = (uint32_t)a[k] < (uint32_t)n && (uint32_t)c[k] < (uint32_t)n;
                bad += (in[k] && !ok) ? 1u : 0u;
                valid[k] = in[k] && ok;
            }
            if (filt) {
                uint32_t wa[kEPT], wc[kEPT];
                bool ha[kEPT], hc[kEPT];
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    ha[k] = hubs && valid[k] && in_hubs(lhub, a[k]);
                    hc[k] = hubs && valid[k] && in_hubs(lhub, c[k]);
                }
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    wa[k] = valid[k] && !ha[k] ? gbits[(uint32_t)a[k] >> 5] : 0xffffffffu;
                    wc[k] = valid[k] && !hc[k] ? gbits[(uint32_t)c[k] >> 5] : 0xffffffffu;
                }
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    const bool both = valid[k] && ((wa[k] >> (a[k] & 31)) & (wc[k] >> (c[k] & 31)) & 1u);
                    nfilt += both ? 1u : 0u;
                    valid[k] = valid[k] && !both;
                }
            }
        };
        sv_segment(len, loader, parent, dst, hdst, write_out != 0, max_link, kept_off, hook_off, nlong, lds, natom,
                   nchase);
    } else {
        const int2* src = in.buf + (int64_t)b * in.cap;
        const int64_t len = in.count[b];
        auto loader = [&](int64_t t0, int32_t* a, int32_t* c, bool* valid) {
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                const int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
                valid[k] = i < len;
                const int2 e = src[valid[k] ? i : 0];
                a[k] = e.x;
                c[k] = e.y;
            }
        };
        sv_segment(len, loader, parent, dst, hdst, write_out != 0, max_link, kept_off, hook_off, nlong, lds, natom,
                   nchase);
    }
    // per-block results (no global atomics on the fast path)
    for (int off = 32; off > 0; off >>= 1) {
        natom += __shfl_xor(natom, off);
        nchase += __shfl_xor(nchase, off);
        nfilt += __shfl_xor(nfilt, off);
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = natom;
        red[1][threadIdx.x >> 6] = nchase;
        red[2][threadIdx.x >> 6] = nfilt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out.count[b] = kept_off;
        hooked_count[b] = hook_off;
        uint32_t sa = 0, sc = 0, sf = 0;
        for (int w = 0; w < kWaves; ++w) {
            sa += red[0][w];
            sc += red[1][w];
            sf += red[2][w];
        }
        segstat[3 * (int64_t)b] = sa;
        segstat[3 * (int64_t)b + 1] = sc;
        segstat[3 * (int64_t)b + 2] = sf;
    }
    if (SOA) {
        // range errors are rare: only then touch a global counter
        for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
        if (lane_id() == 0 && bad) atomic_add_agent(&totals[2], bad);
    }
    // so are finds stopped at the hop bound (totals[4])
    for (int off = 32; off > 0; off >>= 1) nlong += __shfl_xor(nlong, off);
    if (lane_id() == 0 && nlong) atomic_add_agent(&totals[4], nlong);
}

// The largest tree, between two launches of a first pass (after a flatten, so
// every vertex points at its root).  One workgroup samples kPickSamples
// vertices evenly spread over [0, n), counts their roots in an LDS hash table
// and writes the most frequent root (the smallest on ties) to *gflag if it
// holds at least min_count samples, else -1.
constexpr int kPickThreads = 1024;
constexpr int kPickSamples = 4096;
constexpr int kPickSlots = 8192;
__global__ __launch_bounds__(kPickThreads) void giant_pick_kernel(const int32_t* __restrict__ parent, int32_t n,
                                                                  int32_t* __restrict__ gflag, uint32_t min_count) {
    __shared__ int32_t keys[kPickSlots];
    __shared__ uint32_t cnts[kPickSlots];
    __shared__ unsigned long long wbest[kPickThreads / 64];
    for (int i = threadIdx.x; i < kPickSlots; i += kPickThreads) {
        keys[i] = -1;
        cnts[i] = 0;
    }
    __syncthreads();
    for (int j = 0; j < kPickSamples / kPickThreads; ++j) {
        const int64_t i = threadIdx.x + (int64_t)j * kPickThreads;
        const int32_t x = (int32_t)((i * (int64_t)n) / kPickSamples);
        bool root;
        const int32_t r = find_bounded(parent, x, &root);
        if (!root) continue;
        uint32_t h = ((uint32_t)r * 2654435761u) >> 19;   // 13 bits
        for (;;) {
            const int32_t old = atomicCAS(&keys[h], -1, r);
            if (old == -1 || old == r) {
                atomicAdd(&cnts[h], 1u);
                break;
            }
            h = (h + 1) & (kPickSlots - 1);
        }
    }
    __syncthreads();
    // arg-max of (count, smaller root): count in the high word, ~root in the low
    unsigned long long best = 0;
    for (int i = threadIdx.x; i < kPickSlots; i += kPickThreads)
        if (cnts[i]) {
            const unsigned long long k = ((unsigned long long)cnts[i] << 32) | (uint32_t)(~(uint32_t)keys[i]);
            best = k > best ? k : best;
        }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o > best ? o : best;
    }
    if (lane_id() == 0) wbest[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < kPickThreads / 64; ++w) best = wbest[w] > best ? wbest[w] : best;
        const uint32_t cnt = (uint32_t)(best >> 32);
        *gflag = cnt >= min_count ? (int32_t)(~(uint32_t)(best & 0xffffffffull)) : -1;
    }
}

// Bitmap of the tree of *gflag (nothing if it is -1): bit x is set iff
// parent[x] is that tree's root, or x is the root.  Run right after a flatten,
// with no hook in flight, so a set bit means x is in that tree; a vertex left
// short of its root by the flatten's walk bound simply keeps a clear bit.
// One wave covers 64 consecutive vertices and writes two words.  With ids
// (a hub table), the first workgroups (which start first) also write
// tree_ids: ids with every hub whose bit stays clear replaced by -1, one
// bucket per thread.
__global__ __launch_bounds__(kBlock) void giant_bits_kernel(const int32_t* __restrict__ parent, int32_t n,
                                                            const int32_t* __restrict__ gflag,
                                                            uint32_t* __restrict__ bits,
                                                            const int4* __restrict__ ids,
                                                            int4* __restrict__ tree_ids) {
    const int32_t g = *gflag;
    if (g < 0) return;
    bool root;
    const int32_t gr = find_bounded(parent, g, &root);
    if (ids && (int)blockIdx.x < kHubBuckets / kBlock) {
        auto keep = [&](int32_t x) { return x >= 0 && (x == gr || parent[x] == gr) ? x : -1; };
        const int tb = min((int)gridDim.x, kHubBuckets / kBlock);   // workgroups writing the table
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < kHubBuckets; i += tb * kBlock) {
            const int4 q = ids[i];
            tree_ids[i] = make_int4(keep(q.x), keep(q.y), keep(q.z), keep(q.w));
        }
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) & ~(int64_t)63; x0 < n; x0 += stride) {
        const int64_t x = x0 + lane_id();
        const bool in = x < n && (x == gr || parent[x] == gr);
        const uint64_t mk = ballot(in);
        if (lane_id() == 0) *(uint2*)(bits + (x0 >> 5)) = make_uint2((uint32_t)mk, (uint32_t)(mk >> 32));
    }
}

// Hub list: the ids x with deg[x] >= dmin, appended in wave order; at most
// kHubMax are kept (the caller's dmin admits no more).  A wave reads
// kHubU runs of 64 consecutive degrees before it tests any.
constexpr int kHubU = 4;
__global__ __launch_bounds__(kBlock) void hub_list_kernel(const int32_t* __restrict__ deg, int32_t n, int32_t dmin,
                                                          int32_t* __restrict__ list, uint32_t* __restrict__ count) {
    const int64_t per = 64 * kHubU;   // vertices per wave and step
    const int64_t stride = (int64_t)gridDim.x * (kBlock / 64) * per;
    for (int64_t x0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64 * per; x0 < n; x0 += stride) {
        int32_t d[kHubU];
#pragma unroll
        for (int j = 0; j < kHubU; ++j) {
            const int64_t x = x0 + j * 64 + lane_id();
            d[j] = x < n ? deg[x] : 0;
        }
#pragma unroll
        for (int j = 0; j < kHubU; ++j) {
            const bool hub = d[j] >= dmin;   // dmin >= 1, so lanes past n never qualify
            const uint64_t mk = ballot(hub);
            if (mk == 0) continue;
            uint32_t base = 0;
            if (lane_id() == 0) base = atomicAdd(count, (uint32_t)__popcll(mk));
            base = __shfl(base, 0);
            const uint32_t at = base + (uint32_t)__popcll(mk & ((1ull << lane_id()) - 1));
            if (hub && at < (uint32_t)kHubMax) list[at] = (int32_t)(x0 + j * 64 + lane_id());
        }
    }
}

// One workgroup: the hub table of the listed ids (first come, first placed
// in its bucket; a fifth id of a bucket is left out).
constexpr int kHubTableThreads = 1024;
__global__ __launch_bounds__(kHubTableThreads) void hub_table_kernel(const int32_t* __restrict__ list,
                                                                     const uint32_t* __restrict__ count,
                                                                     int4* __restrict__ ids) {
    __shared__ int32_t t[kHubBuckets * 4];
    for (int i = threadIdx.x; i < kHubBuckets * 4; i += kHubTableThreads) t[i] = -1;
    __syncthreads();
    const uint32_t cnt = min(*count, (uint32_t)kHubMax);
    for (uint32_t j = threadIdx.x; j < cnt; j += kHubTableThreads) {
        const int32_t x = list[j];
        int32_t* b = t + 4 * hub_bucket(x);
        for (int k = 0; k < 4; ++k)
            if (atomicCAS(&b[k], -1, x) == -1) break;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHubBuckets; i += kHubTableThreads)
        ids[i] = make_int4(t[4 * i], t[4 * i + 1], t[4 * i + 2], t[4 * i + 3]);
}

// Pointer jumping for the roots hooked in the last pass: each is pointed at
// its current root (or, past kMaxHops links, at the ancestor reached).  Runs
// between passes (no hook in flight).
__global__ __launch_bounds__(kBlock) void sv_shortcut_kernel(int32_t* parent, const int32_t* __restrict__ hooked,
                                                             const uint32_t* __restrict__ hooked_count, int64_t cap) {
    const int b = blockIdx.x;
    const uint32_t cnt = hooked_count[b];
    const int32_t* h = hooked + (int64_t)b * cap;
    for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
        int32_t x = h[j];
        bool root;
        parent[x] = find_bounded(parent, x, &root);
    }
}

// One block: totals[0] = sum of the per-segment survivor counts, totals[1] =
// sum of the per-segment hook counts, totals[3] = the hook counts of segments
// seg_lo .. nseg-1 only (the roots hooked after the last full flatten);
// totals[7..9] = the sums of the segments' atomics, chase reads and edges
// dropped by the bitmap.
constexpr int kTotThreads = 1024;
__global__ __launch_bounds__(kTotThreads) void sv_totals_kernel(const uint32_t* __restrict__ hooked_count,
                                                                const uint32_t* __restrict__ kept_count, int32_t nseg,
                                                                int32_t seg_lo, const uint32_t* __restrict__ segstat,
                                                                unsigned long long* __restrict__ totals) {
    constexpr int W = kTotThreads / 64;
    __shared__ unsigned long long red[6][W];
    unsigned long long sk = 0, sh = 0, sf = 0, s0 = 0, s1 = 0, s2 = 0;
    for (int i = threadIdx.x; i < nseg; i += kTotThreads) {
        s0 += segstat[3 * i];
        s1 += segstat[3 * i + 1];
        s2 += segstat[3 * i + 2];
    }
    // four independent loads in flight per thread
    for (int i0 = threadIdx.x; i0 < nseg; i0 += 4 * kTotThreads) {
        uint32_t a[4], c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + r * kTotThreads;
            a[r] = i < nseg ? kept_count[i] : 0u;
            c[r] = i < nseg ? hooked_count[i] : 0u;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sk += a[r];
            sh += c[r];
            if (i0 + r * kTotThreads >= seg_lo) sf += c[r];
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        sk += __shfl_xor(sk, off);
        sh += __shfl_xor(sh, off);
        sf += __shfl_xor(sf, off);
        s0 += __shfl_xor(s0, off);
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = sk;
        red[1][threadIdx.x >> 6] = sh;
        red[2][threadIdx.x >> 6] = sf;
        red[3][threadIdx.x >> 6] = s0;
        red[4][threadIdx.x >> 6] = s1;
        red[5][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[6] = {};
        for (int w = 0; w < W; ++w)
            for (int k = 0; k < 6; ++k) t[k] += red[k][w];
        totals[0] = t[0];
        totals[1] = t[1];
        totals[3] = t[2];
        totals[7] = t[3];   // atomics issued
        totals[8] = t[4];   // chase reads
        totals[9] = t[5];   // edges dropped by the largest-tree bitmap
    }
}

// Full pointer jumping: every vertex is pointed straight at its root.  Run
// alone (no hook in flight), so the plain stores cannot undo an atomicMin.
// Serves as the final labelling and as the shortcut between the chunks of the
// first pass.
// Flatten round: every vertex is pointed at its root, or, when the root lies
// more than kMaxHops links up, at the ancestor reached, and then *open is set
// (one store per wave).  No hook may run concurrently.  Each round moves every
// vertex of a deep chain at least kMaxHops links up, so depth d takes about
// log(d) / log(kMaxHops) rounds; shallow forests finish in one.
// Each thread walks kFinV vertices up in lock-step (every step issues the
// next read of each unfinished walk before using any), so the dependent
// reads of different walks overlap.
constexpr int kFinV = 4;
__global__ __launch_bounds__(kBlock) void sv_finalize_kernel(int32_t* parent, int32_t n,
                                                             unsigned long long* open) {
    const int64_t stride = (int64_t)gridDim.x * kBlock * kFinV;
    bool left = false;
    for (int64_t b0 = (int64_t)blockIdx.x * kBlock * kFinV + threadIdx.x; b0 < n; b0 += stride) {
        int32_t p[kFinV], q[kFinV], r[kFinV];
        bool act[kFinV];
#pragma unroll
        for (int k = 0; k < kFinV; ++k) {
            const int64_t x = b0 + (int64_t)k * kBlock;
            act[k] = x < n;
            p[k] = act[k] ? parent[x] : 0;
            act[k] = act[k] && p[k] != (int32_t)x;
            q[k] = p[k];
        }
        // q: the vertex reached, r: its parent as read
#pragma unroll
        for (int k = 0; k < kFinV; ++k) r[k] = act[k] ? parent[q[k]] : q[k];
        for (int hop = 0; hop < kMaxHops; ++hop) {
            bool more = false, mv[kFinV];
#pragma unroll
            for (int k = 0; k < kFinV; ++k) {
                mv[k] = act[k] && r[k] != q[k];
                more |= mv[k];
            }
            if (!more) break;
#pragma unroll
            for (int k = 0; k < kFinV; ++k)
                if (mv[k]) q[k] = r[k];
#pragma unroll
            for (int k = 0; k < kFinV; ++k)
                if (mv[k]) r[k] = parent[q[k]];
        }
#pragma unroll
        for (int k = 0; k < kFinV; ++k) {
            if (!act[k]) continue;
            if (q[k] != p[k]) parent[b0 + (int64_t)k * kBlock] = q[k];
            left |= r[k] != q[k];   // stopped at the hop bound short of a root
        }
    }
    if (ballot(left) && lane_id() == 0) __hip_atomic_store(open, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static int grid_for(int64_t n, int per_thread = 1) {
    int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

hipError_t launch_sv_init(int32_t* parent, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    sv_init_kernel<<<grid_for(n, 4), kBlock, 0, s>>>(parent, n);
    return hipGetLastError();
}

hipError_t launch_sv_pass_soa_hubs(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* parent,
                                   SegList out, int32_t seg0, int32_t nblocks, int write_out, int max_link,
                                   int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                                   uint32_t* segstat, const uint32_t* gbits, const int32_t* gflag,
                                   const int4* tree_ids, hipStream_t s) {
    if (seg0 < 0 || nblocks < 1 || seg0 + nblocks > out.nseg) return hipErrorInvalidValue;
    SegList none{nullptr, 0, 0, nullptr};
    if (gbits && gflag)
        sv_pass_kernel<true, true><<<nblocks, kBlock, 0, s>>>(u, v, m, n, seg0, none, parent, out, write_out,
                                                              max_link, hooked, hooked_count, totals, gbits, gflag,
                                                              segstat, tree_ids);
    else
        sv_pass_kernel<true, false><<<nblocks, kBlock, 0, s>>>(u, v, m, n, seg0, none, parent, out, write_out,
                                                               max_link, hooked, hooked_count, totals, nullptr,
                                                               nullptr, segstat, nullptr);
    return hipGetLastError();
}

hipError_t launch_sv_pass_soa(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* parent,
                              SegList out, int32_t seg0, int32_t nblocks, int write_out, int max_link,
                              int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                              uint32_t* segstat, const uint32_t* gbits, const int32_t* gflag, hipStream_t s) {
    return launch_sv_pass_soa_hubs(u, v, m, n, parent, out, seg0, nblocks, write_out, max_link, hooked, hooked_count,
                                   totals, segstat, gbits, gflag, nullptr, s);
}

hipError_t launch_sv_pass_seg(SegList in, int32_t seg0, int32_t nblocks, int32_t* parent, SegList out, int write_out,
                              int max_link, int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                              uint32_t* segstat, hipStream_t s) {
    if (seg0 < 0 || nblocks < 1 || seg0 + nblocks > in.nseg || in.nseg > out.nseg) return hipErrorInvalidValue;
    sv_pass_kernel<false, false><<<nblocks, kBlock, 0, s>>>(nullptr, nullptr, 0, 0, seg0, in, parent, out, write_out,
                                                            max_link, hooked, hooked_count, totals, nullptr, nullptr,
                                                            segstat, nullptr);
    return hipGetLastError();
}

hipError_t launch_giant_pick(const int32_t* parent, int32_t n, int32_t* gflag, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    giant_pick_kernel<<<1, kPickThreads, 0, s>>>(parent, n, gflag, kPickSamples / 16);
    return hipGetLastError();
}

hipError_t launch_giant_bits(const int32_t* parent, int32_t n, const int32_t* gflag, uint32_t* bits, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    giant_bits_kernel<<<grid_for(n, 4), kBlock, 0, s>>>(parent, n, gflag, bits, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_giant_bits_hubs(const int32_t* parent, int32_t n, const int32_t* gflag, uint32_t* bits,
                                  const int4* ids, int4* tree_ids, hipStream_t s) {
    if (n <= 0 || !ids || !tree_ids) return hipErrorInvalidValue;
    giant_bits_kernel<<<grid_for(n, 4), kBlock, 0, s>>>(parent, n, gflag, bits, ids, tree_ids);
    return hipGetLastError();
}

hipError_t launch_hub_list(const int32_t* deg, int32_t n, int32_t dmin, int32_t* list, uint32_t* count, int4* ids,
                           hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    if (dmin < 1) return hipErrorInvalidValue;
    hub_list_kernel<<<grid_for(n, kHubU), kBlock, 0, s>>>(deg, n, dmin, list, count);
    hub_table_kernel<<<1, kHubTableThreads, 0, s>>>(list, count, ids);
    return hipGetLastError();
}

hipError_t launch_sv_shortcut(int32_t* parent, const int32_t* hooked, const uint32_t* hooked_count, int64_t cap,
                              int32_t nseg, hipStream_t s) {
    sv_shortcut_kernel<<<nseg, kBlock, 0, s>>>(parent, hooked, hooked_count, cap);
    return hipGetLastError();
}

hipError_t launch_sv_totals(const uint32_t* hooked_count, const uint32_t* kept_count, int32_t nseg, int32_t seg_lo,
                            const uint32_t* segstat, unsigned long long* totals, hipStream_t s) {
    sv_totals_kernel<<<1, kTotThreads, 0, s>>>(hooked_count, kept_count, nseg, seg_lo, segstat, totals);
    return hipGetLastError();
}

hipError_t launch_sv_finalize(int32_t* parent, int32_t n, unsigned long long* open, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    sv_finalize_kernel<<<grid_for(n, 4), kBlock, 0, s>>>(parent, n, open);
    return hipGetLastError();
}

}  // namespace ccmi
