// Degree distribution (Algorithm 2, first step; Section III-B) and CSR build.
//
// The paper obtains degrees by globally sorting the edge list by source and
// scanning it, then reduces a local array of size c (the maximum degree).  Here
// the same information comes from a bucketed counting pass that keeps every
// counter in LDS:
//
//   A. each block counts, in LDS, the endpoints of its edge chunk per vertex
//      bucket (2^15 consecutive ids);
//   B. a prefix over (bucket, block) gives every block a private output run per
//      bucket;
//   C. each block scatters its endpoints into its runs (LDS cursors,
//      coalesced runs): the 16-bit id within the bucket, and the other end
//      only when a CSR is wanted;
//   D. one block per bucket counts the degrees of its 32768 vertices in LDS,
//      writes deg[], folds the degree histograms (log bins, exact bins below
//      4096, tail list, arg-max) and, when a CSR is wanted, turns the counts
//      into offsets (LDS scan);
//   S, F. (CSR only) the neighbour lists are placed in two steps whose
//      writes stay in LDS-sized windows (see below).
//
// No global atomic touches a per-vertex counter, which matters on MI355X where
// random device-scope atomics run far below the streaming rate.
#include "common.hpp"
#include "degree.hpp"

namespace ccmi {

constexpr int kShift = kBucketShift;
constexpr int kBsz = 1 << kShift;

__device__ __forceinline__ int log_bin(uint32_t d) {
    if (d == 0) return 0;
    int k = 31 - __clz(d);
    int extra = k >= 1 ? (int)((d >> (k - 1)) & 1u) : 0;
    return 1 + 2 * k + extra;
}

__device__ __forceinline__ unsigned long long atomic_max_u64_agent(unsigned long long* p, unsigned long long v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ pass A
// counts[k * nblk + b] = endpoints of block b's edge chunk in bucket k
__device__ __forceinline__ void count_edge(uint32_t* h, int32_t a, int32_t c, int32_t n, uint32_t& bad) {
    if ((uint32_t)a >= (uint32_t)n || (uint32_t)c >= (uint32_t)n) {
        ++bad;
        return;
    }
    atomicAdd(&h[a >> kShift], 1u);
    atomicAdd(&h[c >> kShift], 1u);
}

// VEC: u and v are 16-byte aligned, so the chunk's middle is read as int4
template <bool VEC>
__global__ __launch_bounds__(kBlock) void bucket_count_kernel(const int32_t* __restrict__ u,
                                                              const int32_t* __restrict__ v, int64_t m, int32_t n,
                                                              int64_t chunk, int32_t B, uint32_t* __restrict__ counts,
                                                              unsigned long long* __restrict__ err) {
    extern __shared__ uint32_t h[];
    for (int k = threadIdx.x; k < B; k += kBlock) h[k] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    int64_t end = beg + chunk;
    if (end > m) end = m;
    uint32_t bad = 0;
    int64_t a4 = VEC ? (beg + 3) & ~(int64_t)3 : end;
    if (a4 > end) a4 = end;
    int64_t e4 = VEC ? end & ~(int64_t)3 : end;
    if (e4 < a4) e4 = a4;
    for (int64_t i = beg + threadIdx.x; i < a4; i += kBlock) count_edge(h, u[i], v[i], n, bad);
    for (int64_t i = e4 + threadIdx.x; i < end; i += kBlock) count_edge(h, u[i], v[i], n, bad);
    if (VEC) {
        const int4* u4 = (const int4*)u;
        const int4* v4 = (const int4*)v;
        for (int64_t j = (a4 >> 2) + threadIdx.x; j < (e4 >> 2); j += kBlock) {
            const int4 x = u4[j], y = v4[j];
            count_edge(h, x.x, y.x, n, bad);
            count_edge(h, x.y, y.y, n, bad);
            count_edge(h, x.z, y.z, n, bad);
            count_edge(h, x.w, y.w, n, bad);
        }
    }
    __syncthreads();
    const int nblk = gridDim.x;
    for (int k = threadIdx.x; k < B; k += kBlock) counts[(int64_t)k * nblk + blockIdx.x] = h[k];
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
    if (lane_id() == 0 && bad) atomic_add_agent(err, bad);
}

// one block per bucket k: counts[k][.] -> exclusive prefix over the blocks
// (in place), tot[k] = bucket total.  nblk <= kScanThreads.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void bucket_colscan_kernel(uint32_t* __restrict__ counts, int32_t nblk,
                                                                      unsigned long long* __restrict__ tot) {
    __shared__ uint32_t wsum[kScanThreads / 64 + 1];
    const int k = blockIdx.x, t = threadIdx.x;
    uint32_t* col = counts + (int64_t)k * nblk;
    const uint32_t c = t < nblk ? col[t] : 0u;
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) wsum[t >> 6] = incl;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) { uint32_t q = wsum[w]; wsum[w] = acc; acc += q; }
        wsum[kScanThreads / 64] = acc;
    }
    __syncthreads();
    if (t < nblk) col[t] = wsum[t >> 6] + incl - c;
    if (t == 0) tot[k] = wsum[kScanThreads / 64];
}

// one block per bucket k, from a capped layout's fill counts (runcnt[k][b],
// g scatter blocks of G chunks each): the counted layout's prefix at each
// block's first chunk, prefix[k * nblk + b * G], and tot[k].  The counted
// scatter with the same G reads only those entries.  g <= kScanThreads.
__global__ __launch_bounds__(kScanThreads) void bucket_prefix_from_runs_kernel(
    const uint32_t* __restrict__ runcnt, int32_t g, int32_t G, int32_t nblk, uint32_t* __restrict__ prefix,
    unsigned long long* __restrict__ tot) {
    __shared__ uint32_t wsum[kScanThreads / 64 + 1];
    const int k = blockIdx.x, t = threadIdx.x;
    const uint32_t c = t < g ? runcnt[(int64_t)k * g + t] : 0u;
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) wsum[t >> 6] = incl;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) { uint32_t q = wsum[w]; wsum[w] = acc; acc += q; }
        wsum[kScanThreads / 64] = acc;
    }
    __syncthreads();
    if (t < g) prefix[(int64_t)k * nblk + (int64_t)t * G] = wsum[t >> 6] + incl - c;
    if (t == 0) tot[k] = wsum[kScanThreads / 64];
}

// single block: base[k] = exclusive prefix of tot, base[B] = total
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const unsigned long long* __restrict__ tot, int32_t B,
                                                           unsigned long long* __restrict__ base) {
    __shared__ unsigned long long part[1024];
    const int per = (B + 1023) / 1024;
    const int t = threadIdx.x;
    unsigned long long s = 0;
    for (int j = 0; j < per; ++j) {
        int k = t * per + j;
        if (k < B) s += tot[k];
    }
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over 1024 partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned long long x = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    unsigned long long run = t ? part[t - 1] : 0ull;
    for (int j = 0; j < per; ++j) {
        int k = t * per + j;
        if (k < B) {
            base[k] = run;
            run += tot[k];
        }
    }
    if (t == 1023) base[B] = part[1023];
}

// ------------------------------------------------------------------ pass C
// Bucketed output is structure-of-arrays: loc[i] = endpoint - bucket start
// (16 bits, all the degree count needs), other[i] = the other endpoint
// (written only when a CSR is built).
//
// Each block groups its tile's entries by bucket in LDS, so a bucket's
// entries leave the block as one contiguous run per tile.  Up to kStagedMaxB
// buckets the entries go straight to their buckets (16-bit local ids).  With
// more buckets (n > 2^26) the tile is grouped by super-bucket (kSub = 8
// consecutive buckets, 2^18 vertices) and the entries go, as 18-bit local ids
// in 32-bit words, to the super-bucket's range -- the concatenation of its
// buckets' ranges -- which bucket_split_kernel then splits.  A staged entry
// packs (staging bucket << kKeyShift | local id).
constexpr int kStageThreads = 1024;
constexpr int kCUs = 256;   // compute units of one MI355X (launch sizing only)
constexpr int kSub = 8;
constexpr int kSuperShift = kShift + 3;
// Tile size (measured on MI355X, R-MAT scale 24): one 1024-thread block per
// CU with the longest tile its LDS holds.  Every tile extends each of the
// block's runs (one per bucket) by 2E * 1024 / B entries on average, and with
// a single block per CU the partly written cache lines at the ends of its
// runs stay in the XCD's L2 until the next tiles complete them.  Ids only,
// B = 512: 1.33 ms with 5 edges per thread and two blocks per CU, 1.20 ms
// with 8, 1.13 ms with 12, 1.06 ms with 16 (one block per CU, all three).
// With the other ends (8 bytes of LDS per entry) 8 edges per thread fit.
template <bool OTHER>
struct StageCfg {
    static constexpr int kEdges = OTHER ? 8 : 16;   // edges per thread per tile
    static constexpr int kSlots = kStageThreads * kEdges * 2;
};
static_assert(StageCfg<false>::kSlots <= 65536 && StageCfg<true>::kSlots <= 65536, "ranks are packed in 16 bits");

// Each block walks G consecutive edge chunks (their runs are consecutive in
// the prefix layout, so the cursors simply continue).  The next tile's edges
// are loaded while the current tile is staged and written out.
//
// CAP (degrees only, one level): no count pass runs first.  Block b's run in
// bucket k starts at slot (k * gridDim + b) * cap and holds at most cap
// entries; the block writes how many it filled to runcnt[k * gridDim + b],
// counts the edges with an id outside [0, n) into err[0], and sets err[1]
// if some run would have outgrown cap (from the tile where that happens on,
// the block writes nothing; the caller then runs the counted layout instead).
template <bool OTHER, bool SUPER, bool CAP = false>
__global__ __launch_bounds__(kStageThreads) void bucket_scatter_staged_kernel(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, int64_t m, int32_t n, int64_t chunk, int32_t G,
    int32_t B, int32_t nblk, const uint32_t* __restrict__ prefix, const unsigned long long* __restrict__ base,
    uint16_t* __restrict__ loc, uint32_t* __restrict__ loc32, int32_t* __restrict__ other, uint32_t cap = 0,
    uint32_t* __restrict__ runcnt = nullptr, unsigned long long* __restrict__ err = nullptr) {
    static_assert(!CAP || (!OTHER && !SUPER), "the capped layout is for one-level degree passes");
    constexpr int E = StageCfg<OTHER>::kEdges;
    constexpr int kSh = SUPER ? kSuperShift : kShift;      // staging bucket = id >> kSh
    constexpr int kKeyShift = SUPER ? kSuperShift : 16;    // key = staging bucket << kKeyShift | local
    constexpr uint32_t kLocalMask = (1u << kSh) - 1u;
    constexpr int64_t kTile = (int64_t)kStageThreads * E;
    constexpr uint32_t kJunk = kStagedMaxB + 1;            // toff slot of edges with an id out of range
    constexpr uint32_t kJunkSlot = StageCfg<OTHER>::kSlots;  // their stage slot
    __shared__ uint32_t stage[StageCfg<OTHER>::kSlots + 1];
    __shared__ int32_t stage_o[OTHER ? StageCfg<OTHER>::kSlots + 1 : 1];
    __shared__ uint32_t toff[kStagedMaxB + 2];
    __shared__ uint32_t run[kStagedMaxB];  // next free output slot of each staging bucket
    __shared__ uint32_t rb[kStagedMaxB];   // per tile: output slot of staged slot 0, per staging bucket
    __shared__ uint32_t wsum[kStageThreads / 64];
    __shared__ uint32_t s_full;            // CAP: some run of this block is full
    const int t = threadIdx.x;
    const int c0 = blockIdx.x * G;                         // first edge chunk of this block
    const int NB = SUPER ? (B + kSub - 1) / kSub : B;     // staging buckets (<= 2 * kStageThreads)
    // Thread t owns staging buckets 2t and 2t+1: it alone reads and advances
    // their cursors.  Output positions are below 2m < 2^32 (m < 2^31 is
    // checked by bucket_plan), so 32-bit slot arithmetic is exact.
    auto first_slot = [&](int k) -> uint32_t {
        if (CAP) return ((uint32_t)k * gridDim.x + blockIdx.x) * cap;
        if (SUPER) {
            // chunk c0's first slot in super-bucket k: its first bucket's start
            // plus what the chunks before c0 put into each of its buckets
            const int k0 = k * kSub, k1 = k0 + kSub < B ? k0 + kSub : B;
            unsigned long long r = base[k0];
            for (int q = k0; q < k1; ++q) r += prefix[(int64_t)q * nblk + c0];
            return (uint32_t)r;
        }
        return (uint32_t)(base[k] + prefix[(int64_t)k * nblk + c0]);
    };
    if (2 * t < NB) run[2 * t] = first_slot(2 * t);
    if (2 * t + 1 < NB) run[2 * t + 1] = first_slot(2 * t + 1);
    if (t == 0) s_full = 0;
    const int64_t beg = (int64_t)c0 * chunk;
    int64_t end = beg + (int64_t)G * chunk;
    if (end > m) end = m;
    // the thread's edges of the tile at t0 (-1: past the end); the bound
    // is tested per edge only in a tile that reaches past the end
    int32_t a[E], c[E];
    auto load_tile = [&](int64_t t0) {
        const int32_t* pu = u + (t0 + t);
        const int32_t* pv = v + (t0 + t);
        if (t0 + kTile <= end) {
            // The ids-only scatter streams the edges with non-temporal loads,
            // so they do not push the partly written lines of its runs out of
            // L2 (R-MAT scale 24: 1.54 -> 1.51 ms per degree call); the
            // two-level scatter ran 0.09 ms slower with them.
#pragma unroll
            for (int j = 0; j < E; ++j) {
                if (!OTHER && !SUPER) {
                    a[j] = __builtin_nontemporal_load(pu + j * kStageThreads);
                    c[j] = __builtin_nontemporal_load(pv + j * kStageThreads);
                } else {
                    a[j] = pu[j * kStageThreads];
                    c[j] = pv[j * kStageThreads];
                }
            }
        } else {
            const int64_t rem = end - (t0 + t);   // edge j of the thread is before the end iff j * 1024 < rem
#pragma unroll
            for (int j = 0; j < E; ++j) {
                const bool in = (int64_t)j * kStageThreads < rem;
                a[j] = in ? pu[j * kStageThreads] : -1;
                c[j] = in ? pv[j * kStageThreads] : -1;
            }
        }
    };
    load_tile(beg);
    uint32_t nbad = 0;     // CAP: edges of this thread with an id outside [0, n)
    bool spill = false;    // CAP: an entry did not fit its run
    for (int64_t t0 = beg; t0 < end; t0 += kTile) {
        for (int k = t; k <= NB; k += kStageThreads) toff[k] = 0;
        __syncthreads();
        // rank of each endpoint within its bucket's part of the tile (16 bits
        // each, both ends of edge j packed in r[j]); an edge with an id out
        // of range (or past the end) ranks in the junk slot and stages nothing
        uint32_t r[E];
        uint32_t okm = 0;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const bool ok = (uint32_t)a[j] < (uint32_t)n && (uint32_t)c[j] < (uint32_t)n;
            okm |= ok ? 1u << j : 0u;
            const uint32_t ba = ok ? (uint32_t)a[j] >> kSh : kJunk;
            const uint32_t bc = ok ? (uint32_t)c[j] >> kSh : kJunk;
            r[j] = atomicAdd(&toff[ba], 1u) | (atomicAdd(&toff[bc], 1u) << 16);
            // groups of four edges: eight ranks in flight at a time, and
            // their results live only until packed
            if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
        }
        if (CAP) {
            // edges of this tile before the end, less those in range
            const int64_t rem = end - (t0 + t);
            const int inr = rem <= 0 ? 0
                                     : (rem >= (int64_t)E * kStageThreads ? E
                                                                          : (int)((rem + kStageThreads - 1) / kStageThreads));
            nbad += (uint32_t)(inr - __popc(okm));
        }
        __syncthreads();
        // exclusive scan of the tile's bucket counts (NB <= 2 * 1024 entries)
        {
            const uint32_t n0 = 2 * t < NB ? toff[2 * t] : 0u;
            const uint32_t n1 = 2 * t + 1 < NB ? toff[2 * t + 1] : 0u;
            const uint32_t s = n0 + n1;
            uint32_t incl = s;
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(incl, o);
                if (lane_id() >= o) incl += y;
            }
            if (lane_id() == 63) wsum[t >> 6] = incl;
            __syncthreads();
            if (t == 0) {
                uint32_t acc = 0;
                for (int w = 0; w < kStageThreads / 64; ++w) { uint32_t q = wsum[w]; wsum[w] = acc; acc += q; }
                toff[NB] = acc;
            }
            __syncthreads();
            const uint32_t ex = wsum[t >> 6] + incl - s;
            // staged slot i of bucket k goes to output slot rb[k] + i
            bool full = false;
            if (2 * t < NB) {
                const uint32_t q = run[2 * t];
                toff[2 * t] = ex;
                rb[2 * t] = q - ex;
                run[2 * t] = q + n0;
                if (CAP) full |= q + n0 - first_slot(2 * t) > cap;
            }
            if (2 * t + 1 < NB) {
                const uint32_t q = run[2 * t + 1];
                toff[2 * t + 1] = ex + n0;
                rb[2 * t + 1] = q - (ex + n0);
                run[2 * t + 1] = q + n1;
                if (CAP) full |= q + n1 - first_slot(2 * t + 1) > cap;
            }
            // a full run: nothing more of this block is written (the caller
            // sees err[1] and takes the counted layout)
            if (CAP && full) s_full = 1;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const bool ok = (okm >> j) & 1u;
            const uint32_t ba = ok ? (uint32_t)a[j] >> kSh : kJunk;
            const uint32_t bc = ok ? (uint32_t)c[j] >> kSh : kJunk;
            const uint32_t ka = ((uint32_t)(a[j] >> kSh) << kKeyShift) | ((uint32_t)a[j] & kLocalMask);
            const uint32_t kc = ((uint32_t)(c[j] >> kSh) << kKeyShift) | ((uint32_t)c[j] & kLocalMask);
            const uint32_t sa = ok ? toff[ba] + (r[j] & 0xffffu) : kJunkSlot;
            const uint32_t sc = ok ? toff[bc] + (r[j] >> 16) : kJunkSlot;
            stage[sa] = ka;
            stage[sc] = kc;
            if (OTHER) {
                stage_o[sa] = c[j];
                stage_o[sc] = a[j];
            }
        }
        // the next tile's edges: in flight during the barrier and the write-out
        load_tile(t0 + kTile);
        __syncthreads();
        // contiguous runs per bucket: staged slot i -> its bucket's next free slot
        const uint32_t total = toff[NB];
        if (!CAP || !s_full) {
            for (uint32_t i = t; i < total; i += kStageThreads) {
                const uint32_t q = stage[i];
                const uint32_t pos = rb[q >> kKeyShift] + i;
                if (SUPER) loc32[pos] = q & kLocalMask;
                else loc[pos] = (uint16_t)(q & kLocalMask);
                if (OTHER) other[pos] = stage_o[i];
            }
        }
        __syncthreads();
    }
    if (CAP) {
        // fill counts of this block's runs (thread t owns buckets 2t, 2t + 1)
        for (int k = 2 * t; k < 2 * t + 2 && k < NB; ++k) {
            const uint32_t used = run[k] - first_slot(k);
            runcnt[(int64_t)k * gridDim.x + blockIdx.x] = used < cap ? used : cap;
            spill |= used > cap;
        }
        for (int o = 32; o > 0; o >>= 1) nbad += __shfl_xor(nbad, o);
        if (lane_id() == 0 && nbad) atomic_add_agent(&err[0], (unsigned long long)nbad);
        if (ballot(spill) && lane_id() == 0)
            __hip_atomic_store(&err[1], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Second level for n > 2^26: block S splits super-bucket S (its range is the
// concatenation of buckets 8S .. 8S+7) into those buckets.  A tile of entries
// is grouped by bucket in LDS and each bucket's part leaves as one contiguous
// run.  Ranking is a wave multisplit over the 3-bit bucket index: three
// ballots give every lane the mask of lanes with its bucket, the lowest of
// them reserves the wave's slots with one LDS atomic, and the rank is the
// number of such lanes below.  The next tile is loaded during the write-out.
template <bool OTHER>
struct SplitCfg {
    static constexpr int kE = OTHER ? 8 : 16;   // entries per thread per tile
};
template <bool OTHER>
__global__ __launch_bounds__(kStageThreads) void bucket_split_kernel(const uint32_t* __restrict__ loc32,
                                                                     const int32_t* __restrict__ other32,
                                                                     const unsigned long long* __restrict__ base,
                                                                     int32_t B, uint16_t* __restrict__ loc,
                                                                     int32_t* __restrict__ other) {
    constexpr int E = SplitCfg<OTHER>::kE;
    constexpr uint32_t kNone = 0xffffffffu;   // past the end (local ids have 18 bits)
    __shared__ uint32_t stage[kStageThreads * E];
    __shared__ int32_t stage_o[OTHER ? kStageThreads * E : 1];
    __shared__ uint32_t cnt[kSub + 1];
    __shared__ unsigned long long cur[kSub];
    const int t = threadIdx.x;
    const int k0 = blockIdx.x * kSub;
    const int k1 = k0 + kSub < B ? k0 + kSub : B;
    const unsigned long long beg = base[k0], end = base[k1];
    if (t < kSub) cur[t] = k0 + t < k1 ? base[k0 + t] : 0ull;
    uint32_t q[E];
    int32_t o[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const unsigned long long i = beg + t + (unsigned long long)j * kStageThreads;
        q[j] = i < end ? loc32[i] : kNone;
        o[j] = (OTHER && i < end) ? other32[i] : 0;
    }
    for (unsigned long long t0 = beg; t0 < end; t0 += (unsigned long long)kStageThreads * E) {
        if (t <= kSub) cnt[t] = 0;
        __syncthreads();
        uint32_t rank[E];
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const bool ok = q[j] != kNone;
            const uint32_t sub = ok ? q[j] >> kShift : 0u;
            const uint64_t b0 = ballot(sub & 1u), b1 = ballot(sub & 2u), b2 = ballot(sub & 4u);
            const uint64_t same = ballot(ok) & ((sub & 1u) ? b0 : ~b0) & ((sub & 2u) ? b1 : ~b1) &
                                  ((sub & 4u) ? b2 : ~b2);
            const uint32_t below = lanes_below(same);
            uint32_t r0 = 0;
            if (ok && below == 0) r0 = atomicAdd(&cnt[sub], (uint32_t)__popcll(same));
            r0 = __shfl(r0, __builtin_ctzll(same | (1ull << 63)) & 63);
            rank[j] = r0 + below;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t acc = 0;
            for (int s = 0; s < kSub; ++s) { const uint32_t c = cnt[s]; cnt[s] = acc; acc += c; }
            cnt[kSub] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (q[j] != kNone) {
                const uint32_t slot = cnt[q[j] >> kShift] + rank[j];
                stage[slot] = q[j];
                if (OTHER) stage_o[slot] = o[j];
            }
        // the next tile's entries: in flight during the barrier and the write-out
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const unsigned long long i = t0 + (unsigned long long)kStageThreads * E + t + (unsigned long long)j * kStageThreads;
            q[j] = i < end ? loc32[i] : kNone;
            o[j] = (OTHER && i < end) ? other32[i] : 0;
        }
        __syncthreads();
        const uint32_t total = cnt[kSub];
        for (uint32_t i = t; i < total; i += kStageThreads) {
            const uint32_t x = stage[i];
            const int s = (int)(x >> kShift);
            const unsigned long long pos = cur[s] + (i - cnt[s]);
            loc[pos] = (uint16_t)(x & (kBsz - 1));
            if (OTHER) other[pos] = stage_o[i];
        }
        __syncthreads();
        if (t < kSub) cur[t] += cnt[t + 1] - cnt[t];
        __syncthreads();
    }
}

// h[b] += 1 for every active lane.  Lanes of one wave that share a bin would
// serialise on its LDS counter (every vertex of a lattice has the same
// degree; most R-MAT vertices have degree 0 or 1), so equal bins go through
// one lane: the first lane's bin, then the first remaining lane's bin, then
// one atomic per lane for the rest.  Works for any set of active lanes.
__device__ __forceinline__ void lds_inc_agg(uint32_t* h, uint32_t b) {
    const uint32_t v1 = __builtin_amdgcn_readfirstlane(b);
    const uint64_t m1 = ballot(b == v1);
    if (b == v1) {
        if (lanes_below(m1) == 0) atomicAdd(&h[v1], (uint32_t)__popcll(m1));
    } else {
        const uint32_t v2 = __builtin_amdgcn_readfirstlane(b);
        const uint64_t m2 = ballot(b == v2);
        if (b == v2) {
            if (lanes_below(m2) == 0) atomicAdd(&h[v2], (uint32_t)__popcll(m2));
        } else {
            atomicAdd(&h[b], 1u);
        }
    }
}

// per-vertex histogram update shared by the bucket pass and the standalone kernel
// Degrees >= kExactBins go to the tail list.  A block stages up to kTailLds
// of them in LDS and reserves their slots with one global atomic when it
// flushes; R-MAT scale 24 has about 13 000 such vertices, and one returning
// atomic each on the shared counter serialised chip-wide.
constexpr int kTailLds = 1024;

struct HistLds {
    uint32_t hx[kExactBins];
    uint32_t h64[64];
    unsigned long long best[kBlockD / 64];
    uint32_t tn;                 // tail degrees seen by the block
    unsigned long long tbase;    // first slot the block reserved
    int32_t tbuf[kTailLds];
};

__device__ __forceinline__ void hist_init(HistLds& L, int nthreads) {
    for (int j = threadIdx.x; j < kExactBins; j += nthreads) L.hx[j] = 0;
    if (threadIdx.x < 64) L.h64[threadIdx.x] = 0;
    if (threadIdx.x == 0) L.tn = 0;
}

__device__ __forceinline__ void hist_vertex(HistLds& L, uint32_t d, int32_t x, int32_t* tail, int64_t tail_cap,
                                            unsigned long long* tail_count, unsigned long long& best) {
    if (d < (uint32_t)kExactBins) {
        lds_inc_agg(L.hx, d);   // its log bin is taken from hx[d] at the flush
    } else {
        const uint32_t k = atomicAdd(&L.tn, 1u);
        if (k < (uint32_t)kTailLds) {
            L.tbuf[k] = (int32_t)d;
        } else {
            // past the block's staging: a slot of its own
            unsigned long long slot = atomic_add_agent(tail_count, 1ull);
            if ((int64_t)slot < tail_cap) tail[slot] = (int32_t)d;
        }
        atomicAdd(&L.h64[log_bin(d)], 1u);
    }
    unsigned long long key = ((unsigned long long)d << 32) | (unsigned long long)(~(uint32_t)x);
    best = key > best ? key : best;
}

__device__ __forceinline__ void hist_flush(HistLds& L, unsigned long long best, unsigned long long* hist64,
                                           unsigned long long* histx, unsigned long long* argmax_key, int32_t* tail,
                                           int64_t tail_cap, unsigned long long* tail_count, int nthreads) {
    // the log bins of the degrees below kExactBins, from the exact bins
    for (int d = threadIdx.x; d < kExactBins; d += nthreads)
        if (L.hx[d]) atomicAdd(&L.h64[log_bin((uint32_t)d)], L.hx[d]);
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(best, off);
        best = o > best ? o : best;
    }
    if (lane_id() == 0) L.best[threadIdx.x >> 6] = best;
    // the staged tail degrees: one reservation for the block
    const uint32_t nt = L.tn < (uint32_t)kTailLds ? L.tn : (uint32_t)kTailLds;
    if (threadIdx.x == 0 && nt) L.tbase = atomic_add_agent(tail_count, (unsigned long long)nt);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nt; i += nthreads)
        if ((int64_t)(L.tbase + i) < tail_cap) tail[L.tbase + i] = L.tbuf[i];
    for (int d = threadIdx.x; d < kExactBins; d += nthreads)
        if (L.hx[d]) atomic_add_agent(&histx[d], L.hx[d]);
    if (threadIdx.x < 64 && L.h64[threadIdx.x]) atomic_add_agent(&hist64[threadIdx.x], L.h64[threadIdx.x]);
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < nthreads / 64; ++w) b = L.best[w] > b ? L.best[w] : b;
        if (b) atomic_max_u64_agent(argmax_key, b);
    }
}

// ------------------------------------------------------------------ pass D
constexpr int kUnrollD = 8;
constexpr uint32_t kNoId = 0xffffffffu;   // matches no id of a bucket
// Lanes of one instruction that add to the same LDS counter serialise, and a
// hub can hold a large share of its bucket's entries (over 40% on R-MAT
// scale 24).  So past the kBsz counters each lane has private slots: the
// entries of the block's two hubs (found from a sample) go to slot
// kHubSlots + 64 h + lane, entries that count nowhere (another bucket's, in
// the small-list path) to kJunkSlots + lane.  Every lane of an instruction
// then adds to its own counter for them; the hub slots are folded into the
// hubs' counters at the end.
constexpr int kHubSlots = kBsz;
constexpr int kJunkSlots = kBsz + 128;
constexpr int kCntWords = kBsz + 192;
constexpr int kSampleThreads = 256;   // threads that draw 8 sample ids each
constexpr uint32_t kHubMin = kSampleThreads * 8 / 16;   // a hub holds >= 1/16 of the sample
// Buckets of fewer entries skip the sample (its cost, a few microseconds,
// is what a hub could cost them); so do lists of fewer edges in the
// small-list path, where every block reads the whole list.
constexpr uint64_t kSampleMinEntries = 1u << 17;
constexpr int64_t kSampleMinEdges = 1 << 13;

struct Hubs {
    uint32_t h0 = kNoId, h1 = kNoId;   // hub ids within the bucket (h1 only with h0)
    uint32_t s0, s1, sj;               // this lane's slots
    __device__ Hubs() : s0(kHubSlots + lane_id()), s1(kHubSlots + 64 + lane_id()), sj(kJunkSlots + lane_id()) {}
};

// the counting loops are compiled for 0, 1 and 2 hubs
template <int NH>
struct HubSet {
    Hubs h;
};

template <int NH>
__device__ __forceinline__ uint32_t slot_of(uint32_t x, const HubSet<NH>& hb) {
    uint32_t a = x;
    if constexpr (NH >= 1) a = x == hb.h.h0 ? hb.h.s0 : a;
    if constexpr (NH >= 2) a = x == hb.h.h1 ? hb.h.s1 : a;
    return a;
}

template <int NH>
__device__ __forceinline__ void count_id(uint32_t* cnt, uint32_t x, const HubSet<NH>& hb) {
    atomicAdd(&cnt[slot_of(x, hb)], 1u);
}

// x counts when ok, else it goes to the lane's junk slot
template <int NH>
__device__ __forceinline__ void count_or_junk(uint32_t* cnt, uint32_t x, bool ok, const HubSet<NH>& hb) {
    atomicAdd(&cnt[ok ? slot_of(x, hb) : hb.h.sj], 1u);
}

template <int NH>
__device__ __forceinline__ void count8(uint32_t* cnt, uint4 w, const HubSet<NH>& hb) {
    count_id(cnt, w.x & 0xffffu, hb);
    count_id(cnt, w.x >> 16, hb);
    count_id(cnt, w.y & 0xffffu, hb);
    count_id(cnt, w.y >> 16, hb);
    count_id(cnt, w.z & 0xffffu, hb);
    count_id(cnt, w.z >> 16, hb);
    count_id(cnt, w.w & 0xffffu, hb);
    count_id(cnt, w.w >> 16, hb);
}

// the first `valid` (< 8) entries of an 8-entry group
template <int NH>
__device__ __forceinline__ void count8_masked(uint32_t* cnt, uint4 w, uint32_t valid, const HubSet<NH>& hb) {
    const uint32_t x[8] = {w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16,
                           w.z & 0xffffu, w.z >> 16, w.w & 0xffffu, w.w >> 16};
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if ((uint32_t)e < valid) count_id(cnt, x[e], hb);
}

// f(HubSet<number of hubs>{hb}); the number is uniform over the block
template <class F>
__device__ __forceinline__ void with_hubs(const Hubs& hb, F f) {
    const int nh = __builtin_amdgcn_readfirstlane((int)(hb.h0 != kNoId) + (int)(hb.h1 != kNoId));
    if (nh == 0) f(HubSet<0>{hb});
    else if (nh == 1) f(HubSet<1>{hb});
    else f(HubSet<2>{hb});
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long x, unsigned long long* red) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    if (lane_id() == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long r = 0;
    for (int w = 0; w < kBlockD / 64; ++w) r = red[w] > r ? red[w] : r;
    __syncthreads();
    return r;
}

// The block's hubs: the two most frequent ids of a sample of the bucket's
// entries (sample(t, id) gives thread t < kSampleThreads up to 8 ids, kNoId
// for none), each kept when it holds at least kHubMin of the sample.  Which
// ids are taken changes only how fast the count runs, never its result.
// cnt[0, kBsz) is zero on entry and on return.
template <class F>
__device__ Hubs find_hubs(uint32_t* cnt, unsigned long long* red, F sample) {
    const int t = threadIdx.x;
    uint32_t id[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) id[e] = kNoId;
    if (t < kSampleThreads) sample(t, id);
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (id[e] != kNoId) atomicAdd(&cnt[id[e]], 1u);
    __syncthreads();
    unsigned long long k0 = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (id[e] != kNoId) {
            const unsigned long long key = ((unsigned long long)cnt[id[e]] << 32) | id[e];
            k0 = key > k0 ? key : k0;
        }
    k0 = block_max_u64(k0, red);
    unsigned long long k1 = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (id[e] != kNoId && id[e] != (uint32_t)k0) {
            const unsigned long long key = ((unsigned long long)cnt[id[e]] << 32) | id[e];
            k1 = key > k1 ? key : k1;
        }
    k1 = block_max_u64(k1, red);   // its barriers also end every read of the sample counts
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (id[e] != kNoId) cnt[id[e]] = 0;
    __syncthreads();
    Hubs hb;
    if ((k0 >> 32) >= kHubMin) hb.h0 = (uint32_t)k0;
    if ((k1 >> 32) >= kHubMin) hb.h1 = (uint32_t)k1;
    return hb;
}

constexpr int kMaxRuns = 1024;   // scatter blocks of a capped layout

// runcnt != nullptr: the capped layout of bucket_scatter_staged_kernel<.., CAP>
// (nruns runs of up to cap entries, cap a multiple of 8); base is unused then.
__global__ __launch_bounds__(kBlockD) void bucket_degree_kernel(
    const uint16_t* __restrict__ loc, const unsigned long long* __restrict__ base, int32_t n,
    int32_t* __restrict__ deg, int count_pairs, int want_hist, unsigned long long* __restrict__ hist64,
    unsigned long long* __restrict__ histx, int32_t* __restrict__ tail, int64_t tail_cap,
    unsigned long long* __restrict__ tail_count, unsigned long long* __restrict__ argmax_key, int want_off,
    int64_t* __restrict__ off, uint32_t* __restrict__ gcnt, const uint32_t* __restrict__ runcnt = nullptr,
    int32_t nruns = 0, uint32_t cap = 0, const int32_t* __restrict__ du = nullptr,
    const int32_t* __restrict__ dv = nullptr, int64_t dm = 0, unsigned long long* __restrict__ derr = nullptr) {
    __shared__ uint32_t cnt[kCntWords];   // the bucket's counters, then the lanes' hub and junk slots
    __shared__ uint32_t rp[kMaxRuns + 1];
    __shared__ uint32_t rc[kMaxRuns];
    __shared__ HistLds L;
    __shared__ uint32_t wsum[kBlockD / 64];
    const int k = blockIdx.x;
    const int32_t x0 = k << kShift;
    int32_t nv = n - x0;
    if (nv > kBsz) nv = kBsz;
    for (int j = threadIdx.x; j < kCntWords; j += kBlockD) cnt[j] = 0;
    hist_init(L, kBlockD);
    __syncthreads();
    Hubs hb;
    if (du && count_pairs) {
        // direct (small lists): every block reads the whole edge list and
        // counts the endpoints in its bucket; the others go to the lanes'
        // junk slots.  Block 0 counts the edges with an id outside [0, n).
        if (dm >= kSampleMinEdges) hb = find_hubs(cnt, L.best, [&](int t, uint32_t* id) {
            const int64_t i0 = (dm * t) / kSampleThreads;
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r;
                if (i >= dm) break;
                const int32_t a = du[i], c = dv[i];
                if ((uint32_t)a >= (uint32_t)n || (uint32_t)c >= (uint32_t)n) continue;
                const uint32_t la = (uint32_t)(a - x0), lc = (uint32_t)(c - x0);
                id[2 * r] = la < (uint32_t)nv ? la : kNoId;
                id[2 * r + 1] = lc < (uint32_t)nv ? lc : kNoId;
            }
        });
        uint32_t bad = 0;
        with_hubs(hb, [&](const auto& hs) {
            constexpr int kU = 4;
            for (int64_t i0 = 0; i0 < dm; i0 += (int64_t)kBlockD * kU) {
                int32_t a[kU], c[kU];
#pragma unroll
                for (int r = 0; r < kU; ++r) {
                    const int64_t i = i0 + threadIdx.x + (int64_t)r * kBlockD;
                    a[r] = i < dm ? du[i] : -1;
                    c[r] = i < dm ? dv[i] : -1;
                    if (k == 0 && i < dm && ((uint32_t)a[r] >= (uint32_t)n || (uint32_t)c[r] >= (uint32_t)n)) ++bad;
                }
#pragma unroll
                for (int r = 0; r < kU; ++r) {
                    const bool ok = (uint32_t)a[r] < (uint32_t)n && (uint32_t)c[r] < (uint32_t)n;
                    const uint32_t la = (uint32_t)(a[r] - x0), lc = (uint32_t)(c[r] - x0);
                    count_or_junk(cnt, la, ok && la < (uint32_t)nv, hs);
                    count_or_junk(cnt, lc, ok && lc < (uint32_t)nv, hs);
                }
            }
        });
        for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o);
        if (lane_id() == 0 && bad) atomic_add_agent(derr, (unsigned long long)bad);
    }
    if (runcnt && count_pairs) {
        // capped layout: run r of this bucket is ceil(runcnt / 8) groups of 8
        // entries from group (k * nruns + r) * cap / 8; rp[] is the prefix of
        // those group counts, so group j of the bucket lies in the run r with
        // rp[r] <= j < rp[r + 1]
        const int t = threadIdx.x;
        const uint32_t rcnt = t < nruns ? runcnt[(int64_t)k * nruns + t] : 0u;
        if (t < nruns) rc[t] = rcnt;
        const uint32_t len = (rcnt + 7) / 8;
        uint32_t incl = len;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane_id() >= o) incl += y;
        }
        if (lane_id() == 63) wsum[t >> 6] = incl;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < (t >> 6); ++w) before += wsum[w];
        if (t < nruns) rp[t] = before + incl - len;
        if (t == kBlockD - 1) rp[nruns] = before + incl;   // nruns <= kBlockD: the total
        __syncthreads();
        const uint32_t Q = rp[nruns];
        const uint4* q4 = (const uint4*)loc;
        const uint32_t gpr = cap / 8;   // groups per run slot
        if ((uint64_t)Q * 8 >= kSampleMinEntries) hb = find_hubs(cnt, L.best, [&](int ts, uint32_t* id) {
            // one group at an even spread over the bucket's groups
            const uint32_t j = (uint32_t)(((uint64_t)Q * ts) / kSampleThreads);
            if (j >= Q) return;
            int lo = 0, hi = nruns;   // the last run r with rp[r] <= j
            while (hi - lo > 1) {
                const int mid = (lo + hi) / 2;
                if (rp[mid] <= j) lo = mid;
                else hi = mid;
            }
            const uint32_t within = j - rp[lo];
            const uint32_t c = rc[lo] - within * 8;
            const uint4 w = q4[((uint64_t)k * nruns + lo) * gpr + within];
            const uint32_t x[8] = {w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16,
                                   w.z & 0xffffu, w.z >> 16, w.w & 0xffffu, w.w >> 16};
            for (int e = 0; e < 8; ++e) id[e] = (uint32_t)e < c ? x[e] : kNoId;
        });
        constexpr uint32_t kStep = (uint32_t)kBlockD * kUnrollD;
        // The groups j of a thread only increase, so its run index `cur`
        // only moves forward (runs hold about 500 groups, a thread's j
        // advances by 1024 per slot: a few LDS reads per load).  Only the
        // last group of a run can be partly filled.
        with_hubs(hb, [&](const auto& hs) {
            int cur = 0;
            for (uint32_t j0 = 0; j0 < Q; j0 += kStep) {
                uint4 w[kUnrollD];
                uint32_t nv8[kUnrollD];
#pragma unroll
                for (int r = 0; r < kUnrollD; ++r) {
                    const uint32_t j = j0 + t + (uint32_t)r * kBlockD;
                    w[r] = make_uint4(0, 0, 0, 0);
                    nv8[r] = 0;
                    if (j < Q) {
                        while (rp[cur + 1] <= j) ++cur;   // rp[nruns] = Q > j ends it
                        const uint32_t within = j - rp[cur];
                        const uint32_t c = rc[cur] - within * 8;
                        nv8[r] = c < 8 ? c : 8;
                        w[r] = q4[((uint64_t)k * nruns + cur) * gpr + within];
                    }
                }
#pragma unroll
                for (int r = 0; r < kUnrollD; ++r) {
                    if (nv8[r] == 8) count8(cnt, w[r], hs);
                    else if (nv8[r]) count8_masked(cnt, w[r], nv8[r], hs);
                }
            }
        });
    }
    const bool laid = runcnt || du;   // counted above, not from a counted layout
    const unsigned long long beg = laid ? 0ull : base[k], end = laid ? 0ull : base[k + 1];
    if (!count_pairs) {
        // degrees already known (an earlier pass): only the offsets are wanted
        for (int j = threadIdx.x; j < nv; j += kBlockD) cnt[j] = (uint32_t)deg[x0 + j];
    }
    if (count_pairs && !laid) {
        // 16-byte loads of eight ids between the first and last multiple of 8
        // (loc is 256-byte aligned), kUnrollD of them in flight per thread:
        // one block fills a CU, so the loads in flight must cover HBM latency
        // by themselves.  The few entries outside go one at a time.
        if (end - beg >= kSampleMinEntries) hb = find_hubs(cnt, L.best, [&](int t, uint32_t* id) {
            const unsigned long long i0 = beg + ((end - beg) * (unsigned long long)t) / kSampleThreads;
            for (int e = 0; e < 8; ++e)
                if (i0 + e < end) id[e] = loc[i0 + e];
        });
        const unsigned long long a8 = (beg + 7) & ~7ull, e8 = end & ~7ull;
        with_hubs(hb, [&](const auto& hs) {
            if (a8 >= e8) {
                for (unsigned long long i = beg + threadIdx.x; i < end; i += kBlockD) count_id(cnt, loc[i], hs);
                return;
            }
            for (unsigned long long i = beg + threadIdx.x; i < a8; i += kBlockD) count_id(cnt, loc[i], hs);
            for (unsigned long long i = e8 + threadIdx.x; i < end; i += kBlockD) count_id(cnt, loc[i], hs);
            const uint4* q = (const uint4*)(loc + a8);
            const long long nq = (long long)((e8 - a8) >> 3);
            constexpr long long kStep = (long long)kBlockD * kUnrollD;
            long long j0 = 0;
            for (; j0 + kStep <= nq; j0 += kStep) {
                uint4 w[kUnrollD];
#pragma unroll
                for (int r = 0; r < kUnrollD; ++r) w[r] = q[j0 + threadIdx.x + (long long)r * kBlockD];
#pragma unroll
                for (int r = 0; r < kUnrollD; ++r) count8(cnt, w[r], hs);
            }
            for (long long j = j0 + threadIdx.x; j < nq; j += kBlockD) count8(cnt, q[j], hs);
        });
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // fold the lanes' hub slots into the hubs' counters
        uint32_t c0 = cnt[kHubSlots + threadIdx.x], c1 = cnt[kHubSlots + 64 + threadIdx.x];
        for (int o = 32; o > 0; o >>= 1) {
            c0 += __shfl_xor(c0, o);
            c1 += __shfl_xor(c1, o);
        }
        if (threadIdx.x == 0) {
            if (hb.h0 != kNoId) cnt[hb.h0] += c0;
            if (hb.h1 != kNoId) cnt[hb.h1] += c1;
        }
    }
    __syncthreads();
    unsigned long long best = 0;
    for (int j = threadIdx.x; j < nv && count_pairs; j += kBlockD) {
        uint32_t d = cnt[j];
        deg[x0 + j] = (int32_t)d;
        if (want_hist) hist_vertex(L, d, x0 + j, tail, tail_cap, tail_count, best);
    }
    __syncthreads();
    if (want_hist && count_pairs) hist_flush(L, best, hist64, histx, argmax_key, tail, tail_cap, tail_count, kBlockD);
    if (!want_off) return;
    __syncthreads();
    // exclusive scan of cnt[0..kBsz) in place: 32 entries per thread
    constexpr int per = kBsz / kBlockD;
    const int t = threadIdx.x;
    uint32_t s = 0;
    for (int j = 0; j < per; ++j) s += cnt[t * per + j];
    // wave inclusive scan
    uint32_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) wsum[t >> 6] = incl;
    __syncthreads();
    if (t == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < kBlockD / 64; ++w) { uint32_t q = wsum[w]; wsum[w] = acc; acc += q; }
    }
    __syncthreads();
    uint32_t run = wsum[t >> 6] + incl - s;
    for (int j = 0; j < per; ++j) {
        uint32_t c = cnt[t * per + j];
        cnt[t * per + j] = run;
        run += c;
    }
    __syncthreads();
    for (int j = t; j < nv; j += kBlockD) off[x0 + j] = (int64_t)(beg + cnt[j]);
    if (x0 + nv == n && t == 0) off[n] = (int64_t)end;
    // the CSR fill's per-group counters of this bucket start at zero
    if (gcnt)
        for (int g = t; g < kGroups; g += kBlockD) gcnt[(int64_t)k * kGroups + g] = 0;
}

// ------------------------------------------------------------ CSR fill
// The CSR's rows are filled in two steps, so that every write to adj[] lands
// in a window small enough to assemble in LDS:
//  S. the bucket's entries are regrouped by group of 2^kGrpShift vertices
//     into tmp arrays indexed like adj[] (a group's entries take exactly its
//     rows' slots, [off[x_g], off[x_g + 256]));
//  F. one block per run of groups places each group's entries into an LDS
//     copy of the group's rows and writes the copy out contiguously (groups
//     whose rows exceed the window write straight to adj[]).
constexpr int kGrpV = 1 << kGrpShift;            // vertices per group
constexpr int kGrpE = 8;                         // entries per thread per tile (S)
constexpr int kGrpSlice = 1 << 17;               // about this many entries per block (S)
constexpr int kWcStride = kStageThreads / 64 + 1;   // per-wave group counters, padded against bank conflicts
constexpr int kFillThreads = 1024;
constexpr int kWin = 16384;                      // adjacency entries assembled in LDS (F)
constexpr int kFillU = 4;                        // entries per thread per step (F)

// Rank of this lane's entry among the wave's entries of group g so far (the
// wave's counter for g is wc[g * kWcStride + w]).  Lanes holding the wave's
// candidate group `hot` (wave-uniform; it follows the first valid lane when
// fewer than two lanes held it) reserve together through one lane: a hub can
// put over 40% of its bucket's entries into one group.  Called by all lanes.
__device__ __forceinline__ uint32_t group_rank(uint32_t* wc, int w, uint32_t g, bool ok, uint32_t& hot) {
    const bool h = ok && g == hot;
    const uint64_t m = ballot(h);
    const uint32_t c = (uint32_t)__popcll(m);
    uint32_t r = 0;
    if (c >= 2) {
        const uint32_t below = lanes_below(m);
        if (h && below == 0) r = atomicAdd(&wc[hot * kWcStride + w], c);
        r = __shfl(r, __builtin_ctzll(m));
        if (h) r += below;
        else if (ok) r = atomicAdd(&wc[g * kWcStride + w], 1u);
    } else {
        if (ok) r = atomicAdd(&wc[g * kWcStride + w], 1u);
        const uint64_t am = ballot(ok);
        if (am) hot = __shfl(g, __builtin_ctzll(am));
    }
    return r;
}

// S. Block (k, s) regroups slice s of bucket k (S slices per bucket).  It
// counts the slice's entries per group, reserves that many slots of each
// group's range with one global atomic per group (so slices finish in any
// order and a row's entries are in no fixed order), then places the slice
// tile by tile: entries grouped by (group, wave) in LDS, each group's part of
// the tile written as one run.
__global__ __launch_bounds__(kStageThreads) void csr_group_kernel(const uint16_t* __restrict__ loc,
                                                                  const int32_t* __restrict__ other,
                                                                  const unsigned long long* __restrict__ base,
                                                                  const int64_t* __restrict__ off, int32_t n, int32_t S,
                                                                  uint32_t* __restrict__ gcnt,
                                                                  uint16_t* __restrict__ tloc,
                                                                  int32_t* __restrict__ tother) {
    constexpr int kW = kStageThreads / 64;   // waves
    __shared__ uint16_t sl[kStageThreads * kGrpE];
    __shared__ int32_t so[kStageThreads * kGrpE];
    __shared__ uint32_t wc[kGroups * kWcStride];
    __shared__ uint32_t gstart[kGroups + 1];
    __shared__ uint32_t wsum[kStageThreads / 64];
    __shared__ unsigned long long cur[kGroups];
    const int t = threadIdx.x, w = t >> 6;
    const int k = blockIdx.x / S, sidx = blockIdx.x % S;
    const int64_t x0 = (int64_t)k << kShift;
    const unsigned long long bb = base[k], be = base[k + 1];
    const unsigned long long len = (be - bb + S - 1) / S;
    unsigned long long beg = bb + (unsigned long long)sidx * len;
    if (beg > be) beg = be;
    const unsigned long long end = beg + len < be ? beg + len : be;
    uint32_t hot = 0xffffffffu;   // no group index matches it
    // 1. the slice's entries per group: 16-byte loads of eight ids between the
    //    first and last multiple of 8 (loc is 256-byte aligned), the rest one by one
    for (int i = t; i < kGroups * kWcStride; i += kStageThreads) wc[i] = 0;
    __syncthreads();
    {
        const unsigned long long a8 = (beg + 7) & ~7ull, e8 = end & ~7ull;
        if (a8 >= e8) {
            for (unsigned long long i = beg + t; i < end; i += kStageThreads)
                atomicAdd(&wc[(loc[i] >> kGrpShift) * kWcStride + w], 1u);
        } else {
            for (unsigned long long i = beg + t; i < a8; i += kStageThreads)
                atomicAdd(&wc[(loc[i] >> kGrpShift) * kWcStride + w], 1u);
            for (unsigned long long i = e8 + t; i < end; i += kStageThreads)
                atomicAdd(&wc[(loc[i] >> kGrpShift) * kWcStride + w], 1u);
            const uint4* q4 = (const uint4*)(loc + a8);
            const long long nq = (long long)((e8 - a8) >> 3);
            for (long long j0 = 0; j0 < nq; j0 += 2 * kStageThreads) {   // uniform trip count
                uint4 x[2];
                bool okx[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const long long j = j0 + t + (long long)r * kStageThreads;
                    okx[r] = j < nq;
                    x[r] = okx[r] ? q4[j] : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const uint32_t wv[4] = {x[r].x, x[r].y, x[r].z, x[r].w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        (void)group_rank(wc, w, (wv[h] & 0xffffu) >> kGrpShift, okx[r], hot);
                        (void)group_rank(wc, w, wv[h] >> (16 + kGrpShift), okx[r], hot);
                    }
                }
            }
        }
    }
    __syncthreads();
    // 2. reserve the slice's slots in each group's range
    if (t < kGroups) {
        uint32_t c = 0;
        for (int q = 0; q < kW; ++q) c += wc[t * kWcStride + q];
        const int64_t x = x0 + ((int64_t)t << kGrpShift);
        unsigned long long r = 0;
        if (c) r = __hip_atomic_fetch_add(&gcnt[(int64_t)k * kGroups + t], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cur[t] = (x < n ? (unsigned long long)off[x] : be) + r;
    }
    __syncthreads();
    // 3. place the slice
    for (unsigned long long t0 = beg; t0 < end; t0 += (unsigned long long)kStageThreads * kGrpE) {
        for (int i = t; i < kGroups * kWcStride; i += kStageThreads) wc[i] = 0;
        __syncthreads();
        uint32_t q[kGrpE], rank[kGrpE];
        int32_t o[kGrpE];
        bool ok[kGrpE];
#pragma unroll
        for (int j = 0; j < kGrpE; ++j) {
            const unsigned long long i = t0 + t + (unsigned long long)j * kStageThreads;
            ok[j] = i < end;
            q[j] = ok[j] ? loc[i] : 0u;
            o[j] = ok[j] ? other[i] : 0;
        }
#pragma unroll
        for (int j = 0; j < kGrpE; ++j) rank[j] = group_rank(wc, w, q[j] >> kGrpShift, ok[j], hot);
        __syncthreads();
        // exclusive scan of the (group, wave) counts in group-major order
        // (2 entries per thread, both of one group)
        {
            const int g = (2 * t) / kW, wv = (2 * t) % kW;
            const uint32_t c0 = wc[g * kWcStride + wv], c1 = wc[g * kWcStride + wv + 1], sm = c0 + c1;
            uint32_t incl = sm;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d);
                if (lane_id() >= d) incl += y;
            }
            if (lane_id() == 63) wsum[w] = incl;
            __syncthreads();
            if (t == 0) {
                uint32_t acc = 0;
                for (int i = 0; i < kStageThreads / 64; ++i) { const uint32_t c = wsum[i]; wsum[i] = acc; acc += c; }
                gstart[kGroups] = acc;
            }
            __syncthreads();
            const uint32_t ex = wsum[w] + incl - sm;
            wc[g * kWcStride + wv] = ex;
            wc[g * kWcStride + wv + 1] = ex + c0;
        }
        __syncthreads();
        if (t < kGroups) gstart[t] = wc[t * kWcStride];
#pragma unroll
        for (int j = 0; j < kGrpE; ++j)
            if (ok[j]) {
                const uint32_t slot = wc[(q[j] >> kGrpShift) * kWcStride + w] + rank[j];
                sl[slot] = (uint16_t)q[j];
                so[slot] = o[j];
            }
        __syncthreads();
        const uint32_t total = gstart[kGroups];
        for (uint32_t i = t; i < total; i += kStageThreads) {
            const int g = sl[i] >> kGrpShift;
            const unsigned long long pos = cur[g] + (i - gstart[g]);
            tloc[pos] = sl[i];
            tother[pos] = so[i];
        }
        __syncthreads();
        if (t < kGroups) cur[t] += gstart[t + 1] - gstart[t];
        __syncthreads();
    }
}

// Reserves the next slot of row xl for each lane; lanes of a wave that share
// the wave's first row (a hub) take consecutive slots with one LDS atomic.
__device__ __forceinline__ uint32_t row_slot(uint32_t* cur, bool ok, int32_t xl) {
    const int first = __builtin_ctzll(ballot(ok) | (1ull << 63)) & 63;
    const int32_t lead = __shfl(xl, first);
    const uint64_t same = ballot(ok && xl == lead);
    const uint32_t rank = lanes_below(same);
    uint32_t basepos = 0;
    if (ok && xl == lead && rank == 0) basepos = atomicAdd(&cur[lead], (uint32_t)__popcll(same));
    basepos = __shfl(basepos, __builtin_ctzll(same | (1ull << 63)) & 63);
    if (!ok) return 0;
    return xl == lead ? basepos + rank : atomicAdd(&cur[xl], 1u);
}

__global__ __launch_bounds__(kFillThreads) void csr_fill_kernel(const uint16_t* __restrict__ tloc,
                                                                const int32_t* __restrict__ tother,
                                                                const int64_t* __restrict__ off, int32_t n,
                                                                int64_t ngroups, int32_t gpb,
                                                                int32_t* __restrict__ adj) {
    __shared__ int32_t win[kWin];
    __shared__ uint32_t cur[kGrpV];
    __shared__ int64_t offs[kGrpV + 1];
    const int t = threadIdx.x;
    for (int64_t G = (int64_t)blockIdx.x * gpb; G < ngroups && G < (int64_t)(blockIdx.x + 1) * gpb; ++G) {
        const int64_t xs = G << kGrpShift;
        const int64_t xe = xs + kGrpV < n ? xs + kGrpV : n;
        const int nv = (int)(xe - xs);
        __syncthreads();   // the previous group is done with offs, cur and win
        for (int j = t; j <= nv; j += kFillThreads) offs[j] = off[xs + j];
        for (int j = t; j < kGrpV; j += kFillThreads) cur[j] = 0;
        __syncthreads();
        const int64_t a = offs[0], b = offs[nv];
        const bool staged = b - a <= kWin;   // block-uniform
        // kFillU entries per thread per step, loaded before any is placed
        for (int64_t i0 = a; i0 < b; i0 += (int64_t)kFillThreads * kFillU) {
            int32_t xl[kFillU], y[kFillU];
            bool ok[kFillU];
#pragma unroll
            for (int u = 0; u < kFillU; ++u) {
                const int64_t i = i0 + t + (int64_t)u * kFillThreads;
                ok[u] = i < b;
                xl[u] = ok[u] ? (int32_t)(tloc[i] & (kGrpV - 1)) : 0;
                y[u] = ok[u] ? tother[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < kFillU; ++u) {
                const uint32_t r = row_slot(cur, ok[u], xl[u]);
                if (ok[u]) {
                    if (staged) win[offs[xl[u]] - a + r] = y[u];
                    else adj[offs[xl[u]] + r] = y[u];
                }
            }
        }
        if (staged) {
            __syncthreads();
            for (int64_t i = t; i < b - a; i += kFillThreads) adj[a + i] = win[i];
        }
    }
}

// --------------------------------------------- standalone histogram kernel
__global__ __launch_bounds__(kBlockD) void degree_hist_kernel(const int32_t* __restrict__ deg, int32_t n,
                                                              unsigned long long* __restrict__ hist64,
                                                              unsigned long long* __restrict__ histx,
                                                              int32_t* __restrict__ tail, int64_t tail_cap,
                                                              unsigned long long* __restrict__ tail_count,
                                                              unsigned long long* __restrict__ argmax_key) {
    __shared__ HistLds L;
    hist_init(L, kBlockD);
    __syncthreads();
    unsigned long long best = 0;
    for (int64_t x = (int64_t)blockIdx.x * kBlockD + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlockD)
        hist_vertex(L, (uint32_t)deg[x], (int32_t)x, tail, tail_cap, tail_count, best);
    __syncthreads();
    hist_flush(L, best, hist64, histx, argmax_key, tail, tail_cap, tail_count, kBlockD);
}

// ------------------------------------------------------------------ host
int bucket_plan(int32_t n, int64_t m, BucketPlan* p) {
    p->B = (int32_t)(((int64_t)n + kBsz - 1) >> kShift);
    if (p->B < 1) p->B = 1;
    if (p->B > kMaxBuckets) return -1;
    if (m < 0 || m >= ((int64_t)1 << 31)) return -1;   // 32-bit prefixes and output slots
    int64_t nblk = (m + 65535) / 65536;   // ~64K edges per block chunk
    if (nblk < 1) nblk = 1;
    if (nblk > kScanThreads) nblk = kScanThreads;
    p->nblk = (int32_t)nblk;
    p->chunk = (m + nblk - 1) / nblk;
    if (p->chunk < 1) p->chunk = 1;
    return 0;
}

template <bool OTHER>
static void scatter_with(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                         const BucketBufs& w, hipStream_t s) {
    // chunks per block: about one block per CU once there are enough chunks
    const int G = p.nblk >= 2 * kCUs ? p.nblk / kCUs : 1;
    const int grid = (p.nblk + G - 1) / G;
    if (p.B <= kStagedMaxB) {
        bucket_scatter_staged_kernel<OTHER, false><<<grid, kStageThreads, 0, s>>>(
            u, v, m, n, p.chunk, G, p.B, p.nblk, w.counts, w.base, w.loc, nullptr, OTHER ? w.other : nullptr);
    } else {
        bucket_scatter_staged_kernel<OTHER, true><<<grid, kStageThreads, 0, s>>>(
            u, v, m, n, p.chunk, G, p.B, p.nblk, w.counts, w.base, nullptr, w.loc32, OTHER ? w.other32 : nullptr);
        bucket_split_kernel<OTHER><<<(p.B + kSub - 1) / kSub, kStageThreads, 0, s>>>(
            w.loc32, OTHER ? w.other32 : nullptr, w.base, p.B, w.loc, OTHER ? w.other : nullptr);
    }
}

static hipError_t launch_scatter(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                 const BucketBufs& w, bool with_other, hipStream_t s) {
    if (with_other) scatter_with<true>(u, v, m, n, p, w, s);
    else scatter_with<false>(u, v, m, n, p, w, s);
    return hipGetLastError();
}

// steps S and F of the CSR fill (offsets already in off[])
static hipError_t launch_csr_fill(int64_t m, int32_t n, const BucketPlan& p, const BucketBufs& w, const int64_t* off,
                                  int32_t* adj, hipStream_t s) {
    // slices per bucket: about kGrpSlice entries each
    int64_t S = (2 * m / p.B + kGrpSlice - 1) / kGrpSlice;
    if (S < 1) S = 1;
    if (S > 64) S = 64;
    csr_group_kernel<<<(unsigned)(p.B * S), kStageThreads, 0, s>>>(w.loc, w.other, w.base, off, n, (int32_t)S, w.gcnt,
                                                                   w.tloc, w.tother);
    const int64_t ngroups = ((int64_t)n + kGrpV - 1) >> kGrpShift;
    // runs of groups per block: about one LDS window of entries each
    const int64_t avg = ngroups > 0 ? (2 * m) / ngroups : 0;
    int gpb = 1;
    while (gpb < 64 && (int64_t)gpb * 2 * avg <= kWin) gpb *= 2;
    const int64_t grid = (ngroups + gpb - 1) / gpb;
    csr_fill_kernel<<<(unsigned)grid, kFillThreads, 0, s>>>(w.tloc, w.tother, off, n, ngroups, gpb, adj);
    return hipGetLastError();
}

// Lists this small take the direct count (every bucket's block reads all of
// the edges: at most 4 x 2 MB) and the direct CSR.
constexpr int kDirectMaxB = 4;
constexpr int64_t kDirectMaxM = (int64_t)1 << 18;

// CSR of a small list in one launch (degrees known): block k owns bucket k.
// It sums the degrees below its bucket, scans its bucket's degrees in LDS
// into row cursors (writing off[]), then reads every edge and places the
// endpoints in its bucket through those cursors (returning LDS atomics).
// Rows come out in no particular order, as the contract allows.
__global__ __launch_bounds__(kBlockD) void csr_direct_kernel(const int32_t* __restrict__ u,
                                                             const int32_t* __restrict__ v, int64_t m, int32_t n,
                                                             const int32_t* __restrict__ deg,
                                                             int64_t* __restrict__ off, int32_t* __restrict__ adj) {
    __shared__ uint32_t cur[kBsz];
    __shared__ unsigned long long wred[kBlockD / 64];
    __shared__ uint32_t wsum[kBlockD / 64];
    const int k = blockIdx.x, t = threadIdx.x;
    const int32_t x0 = k << kShift;
    int32_t nv = n - x0;
    if (nv > kBsz) nv = kBsz;
    // degrees of the vertices below this bucket
    unsigned long long below = 0;
    for (int32_t x = t; x < x0; x += kBlockD) below += (unsigned long long)deg[x];
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
    if (lane_id() == 0) wred[t >> 6] = below;
    // exclusive scan of this bucket's degrees: coalesced loads into LDS,
    // then 32 consecutive entries per thread
    constexpr int per = kBsz / kBlockD;
#pragma unroll 8
    for (int j = 0; j < per; ++j) {
        const int32_t x = t + j * kBlockD;
        cur[x] = x < nv ? (uint32_t)deg[x0 + x] : 0u;
    }
    __syncthreads();
    uint32_t d[per], sum = 0;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        d[j] = cur[t * per + j];
        sum += d[j];
    }
    uint32_t incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) wsum[t >> 6] = incl;
    __syncthreads();   // also: every thread has read its degrees from cur[] before they are overwritten
    unsigned long long base = 0;
    uint32_t before = 0, total = 0;
    for (int w = 0; w < kBlockD / 64; ++w) {
        base += wred[w];
        if (w < (t >> 6)) before += wsum[w];
        total += wsum[w];
    }
    uint32_t run = before + incl - sum;
#pragma unroll
    for (int j = 0; j < per; ++j) {
        const int32_t x = t * per + j;
        cur[x] = run;
        if (x < nv) off[x0 + x] = (int64_t)(base + run);
        run += d[j];
    }
    if (x0 + nv == n && t == 0) off[n] = (int64_t)(base + total);
    __syncthreads();
    int32_t* row = adj + base;   // this bucket's rows, relative to its first
    // eight edges' reads in flight per thread, then their placements
    constexpr int kU = 8;
    for (int64_t i0 = 0; i0 < m; i0 += (int64_t)kBlockD * kU) {
        int32_t a[kU], c[kU];
#pragma unroll
        for (int r = 0; r < kU; ++r) {
            const int64_t i = i0 + t + (int64_t)r * kBlockD;
            a[r] = i < m ? u[i] : -1;
            c[r] = i < m ? v[i] : -1;
        }
#pragma unroll
        for (int r = 0; r < kU; ++r) {
            const uint32_t la = (uint32_t)(a[r] - x0), lc = (uint32_t)(c[r] - x0);
            if (a[r] >= 0 && la < (uint32_t)nv) row[atomicAdd(&cur[la], 1u)] = c[r];
            if (c[r] >= 0 && lc < (uint32_t)nv) row[atomicAdd(&cur[lc], 1u)] = a[r];
        }
    }
}


static void count_and_scan(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                           BucketBufs& w, hipStream_t s);

hipError_t launch_bucket_csr_from_deg(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                      BucketBufs& w, int32_t* deg, int64_t* off, int32_t* adj, hipStream_t s) {
    if (p.B <= kDirectMaxB && m <= kDirectMaxM) {
        csr_direct_kernel<<<p.B, kBlockD, 0, s>>>(u, v, m, n, deg, off, adj);
        return hipGetLastError();
    }
    if (!w.counted) {
        // The degree pass used the capped layout.  Its fill counts are the
        // counted layout's per-block counts (the same blocks read the same
        // edges), so their scan replaces a second count over the edge list;
        // the prefixes go to the CSR fill's scratch, unused until the fill.
        // Without that scratch, count and scan again (the ids were checked
        // then; the error counter only grows).
        const int G = p.nblk >= 2 * kCUs ? p.nblk / kCUs : 1;
        if (w.capped_grid > 0 && w.capped_grid == (p.nblk + G - 1) / G && w.tloc &&
            (size_t)p.B * p.nblk * sizeof(uint32_t) <= (size_t)2 * m * sizeof(uint16_t)) {
            uint32_t* prefix = (uint32_t*)w.tloc;
            bucket_prefix_from_runs_kernel<<<p.B, kScanThreads, 0, s>>>(w.counts, w.capped_grid, G, p.nblk, prefix,
                                                                         w.tot);
            bucket_scan_kernel<<<1, 1024, 0, s>>>(w.tot, p.B, w.base);
            w.counts = prefix;
            w.counted = true;
        } else {
            count_and_scan(u, v, m, n, p, w, s);
        }
        w.capped_grid = 0;
        w.other_written = false;
    }
    if (!w.other_written) {
        // the degree pass kept only the local ids: scatter again with the
        // other endpoints.  Both arrays are rewritten together, because the
        // order inside a tile's run is not reproducible between launches.
        hipError_t e = launch_scatter(u, v, m, n, p, w, true, s);
        if (e != hipSuccess) return e;
        w.other_written = true;
    }
    bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(w.loc, w.base, n, deg, 0, 0, nullptr, nullptr, nullptr, 0, nullptr,
                                                  nullptr, 1, off, w.gcnt);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_csr_fill(m, n, p, w, off, adj, s);
}

// Grid and run capacity of the capped layout, or false when it does not
// apply: CSR builds and two-level passes take the counted layout, and so do
// lists whose capped runs would not fit the loc buffer or 32-bit slots.  A
// run holds twice its bucket's average share of the block's endpoints plus
// 256: a hub of a third of its bucket's entries still fits.
static bool capped_plan(int64_t m, const BucketPlan& p, const BucketBufs& w, int* grid, uint32_t* cap) {
    if (p.B > kStagedMaxB || m < ((int64_t)1 << 16)) return false;
    const int G = p.nblk >= 2 * kCUs ? p.nblk / kCUs : 1;
    const int g = (p.nblk + G - 1) / G;
    if (g > kMaxRuns) return false;
    const int64_t per_block = 2 * (int64_t)G * p.chunk;   // endpoints of a block's edges (at most)
    const int64_t c = ((2 * per_block / p.B + 256) + 7) & ~(int64_t)7;
    const int64_t slots = (int64_t)g * p.B * c;
    if (slots + per_block >= ((int64_t)1 << 32) || slots > w.loc_cap) return false;   // 32-bit slot arithmetic
    *grid = g;
    *cap = (uint32_t)c;
    return true;
}

// pass A and the prefixes of the counted layout
static void count_and_scan(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                           BucketBufs& w, hipStream_t s) {
    const size_t lds = (size_t)p.B * sizeof(uint32_t);
    if ((((uintptr_t)u | (uintptr_t)v) & 15) == 0)
        bucket_count_kernel<true><<<p.nblk, kBlock, lds, s>>>(u, v, m, n, p.chunk, p.B, w.counts, w.err);
    else
        bucket_count_kernel<false><<<p.nblk, kBlock, lds, s>>>(u, v, m, n, p.chunk, p.B, w.counts, w.err);
    bucket_colscan_kernel<<<p.B, kScanThreads, 0, s>>>(w.counts, p.nblk, w.tot);
    bucket_scan_kernel<<<1, 1024, 0, s>>>(w.tot, p.B, w.base);
    w.counted = true;
    w.capped_grid = 0;
}

hipError_t launch_bucket_degree(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                BucketBufs& w, int32_t* deg, int want_hist, unsigned long long* hist64,
                                unsigned long long* histx, int32_t* tail, int64_t tail_cap,
                                unsigned long long* tail_count, unsigned long long* argmax_key, int want_csr,
                                int64_t* off, int32_t* adj, hipStream_t s, bool allow_capped) {
    int grid = 0;
    uint32_t cap = 0;
    if (p.B <= kDirectMaxB && m <= kDirectMaxM) {
        // small lists: each bucket's block counts straight from the edges
        // (one launch), and a CSR takes one more
        w.counted = false;
        w.other_written = false;
        w.capped_grid = 0;
        bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(nullptr, nullptr, n, deg, 1, want_hist, hist64, histx, tail,
                                                      tail_cap, tail_count, argmax_key, 0, nullptr, nullptr, nullptr,
                                                      0, 0, u, v, m, w.err);
        if (want_csr) csr_direct_kernel<<<p.B, kBlockD, 0, s>>>(u, v, m, n, deg, off, adj);
        return hipGetLastError();
    }
    if (allow_capped && !want_csr && capped_plan(m, p, w, &grid, &cap)) {
        // no count pass: each scatter block fills runs of fixed capacity
        const int G = p.nblk >= 2 * kCUs ? p.nblk / kCUs : 1;
        bucket_scatter_staged_kernel<false, false, true><<<grid, kStageThreads, 0, s>>>(
            u, v, m, n, p.chunk, G, p.B, p.nblk, nullptr, nullptr, w.loc, nullptr, nullptr, cap, w.counts, w.err);
        w.counted = false;
        w.other_written = false;
        w.capped_grid = grid;
        bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(w.loc, nullptr, n, deg, 1, want_hist, hist64, histx, tail,
                                                      tail_cap, tail_count, argmax_key, 0, nullptr, nullptr,
                                                      w.counts, grid, cap);
        return hipGetLastError();
    }
    const size_t lds = (size_t)p.B * sizeof(uint32_t);
    (void)lds;
    count_and_scan(u, v, m, n, p, w, s);
    hipError_t e = launch_scatter(u, v, m, n, p, w, want_csr != 0, s);
    if (e != hipSuccess) return e;
    w.other_written = want_csr != 0;
    bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(w.loc, w.base, n, deg, 1, want_hist, hist64, histx, tail, tail_cap,
                                                  tail_count, argmax_key, want_csr, off, want_csr ? w.gcnt : nullptr);
    e = hipGetLastError();
    if (e != hipSuccess || !want_csr) return e;
    return launch_csr_fill(m, n, p, w, off, adj, s);
}

hipError_t launch_degree_hist(const int32_t* deg, int32_t n, unsigned long long* hist64, unsigned long long* histx,
                              int32_t* tail, int64_t tail_cap, unsigned long long* tail_count,
                              unsigned long long* argmax_key, hipStream_t s) {
    int64_t g = ((int64_t)n + kBlockD * 8 - 1) / (kBlockD * 8);
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    degree_hist_kernel<<<(int)g, kBlockD, 0, s>>>(deg, n, hist64, histx, tail, tail_cap, tail_count, argmax_key);
    return hipGetLastError();
}

}  // namespace ccmi
