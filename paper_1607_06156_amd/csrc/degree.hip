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
//   C. each block scatters (endpoint, other end) pairs into its runs (LDS
//      cursors, coalesced runs);
//   D. one block per bucket counts the degrees of its 32768 vertices in LDS,
//      writes deg[], folds the degree histograms (log bins, exact bins below
//      4096, tail list, arg-max) and, when a CSR is wanted, turns the counts
//      into offsets (LDS scan) and scatters the neighbour lists into the
//      bucket's contiguous adjacency range.
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
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
        int32_t a = u[i], c = v[i];
        if ((uint32_t)a >= (uint32_t)n || (uint32_t)c >= (uint32_t)n) {
            ++bad;
            continue;
        }
        atomicAdd(&h[a >> kShift], 1u);
        atomicAdd(&h[c >> kShift], 1u);
    }
    __syncthreads();
    uint32_t* row = counts + (int64_t)blockIdx.x * B;
    for (int k = threadIdx.x; k < B; k += kBlock) row[k] = h[k];
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
    if (lane_id() == 0 && bad) atomic_add_agent(err, bad);
}

// column totals: tot[k] = sum_b counts[b][k]
__global__ __launch_bounds__(kBlock) void bucket_totals_kernel(const uint32_t* __restrict__ counts, int32_t nblk,
                                                               int32_t B, unsigned long long* __restrict__ tot) {
    int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= B) return;
    unsigned long long s = 0;
    for (int b = 0; b < nblk; ++b) s += counts[(int64_t)b * B + k];
    tot[k] = s;
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

// offs[b][k] = base[k] + sum_{b' < b} counts[b'][k]
__global__ __launch_bounds__(kBlock) void bucket_offsets_kernel(const uint32_t* __restrict__ counts, int32_t nblk,
                                                                int32_t B, const unsigned long long* __restrict__ base,
                                                                unsigned long long* __restrict__ offs) {
    int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= B) return;
    unsigned long long run = base[k];
    for (int b = 0; b < nblk; ++b) {
        offs[(int64_t)b * B + k] = run;
        run += counts[(int64_t)b * B + k];
    }
}

// ------------------------------------------------------------------ pass C
__global__ __launch_bounds__(kBlock) void bucket_scatter_kernel(const int32_t* __restrict__ u,
                                                                const int32_t* __restrict__ v, int64_t m, int32_t n,
                                                                int64_t chunk, int32_t B,
                                                                const unsigned long long* __restrict__ offs,
                                                                int2* __restrict__ pairs) {
    extern __shared__ uint32_t cur[];
    for (int k = threadIdx.x; k < B; k += kBlock) cur[k] = 0;
    __syncthreads();
    const unsigned long long* row = offs + (int64_t)blockIdx.x * B;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    int64_t end = beg + chunk;
    if (end > m) end = m;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
        int32_t a = u[i], c = v[i];
        if ((uint32_t)a >= (uint32_t)n || (uint32_t)c >= (uint32_t)n) continue;
        uint32_t pa = atomicAdd(&cur[a >> kShift], 1u);
        pairs[row[a >> kShift] + pa] = make_int2(a, c);
        uint32_t pc = atomicAdd(&cur[c >> kShift], 1u);
        pairs[row[c >> kShift] + pc] = make_int2(c, a);
    }
}

// Same scatter with the tile's pairs first grouped by bucket in LDS, so each
// bucket's pairs leave the block as one contiguous run per tile (for B up to
// kStagedMaxB buckets).
constexpr int kStageThreads = 1024;
constexpr int kStageEdges = 3;                         // edges per thread per tile (LDS: 2 blocks/CU)
constexpr int kStagePairs = kStageThreads * kStageEdges * 2;

__global__ __launch_bounds__(kStageThreads) void bucket_scatter_staged_kernel(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, int64_t m, int32_t n, int64_t chunk, int32_t B,
    const unsigned long long* __restrict__ offs, int2* __restrict__ pairs) {
    __shared__ int2 stage[kStagePairs];
    __shared__ uint32_t toff[kStagedMaxB + 1];
    __shared__ uint32_t run[kStagedMaxB];
    __shared__ uint32_t wsum[kStageThreads / 64];
    const int t = threadIdx.x;
    for (int k = t; k < B; k += kStageThreads) run[k] = 0;
    const unsigned long long* row = offs + (int64_t)blockIdx.x * B;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    int64_t end = beg + chunk;
    if (end > m) end = m;
    for (int64_t t0 = beg; t0 < end; t0 += (int64_t)kStageThreads * kStageEdges) {
        for (int k = t; k <= B; k += kStageThreads) toff[k] = 0;
        __syncthreads();
        int2 p[2 * kStageEdges];
        uint32_t rank[2 * kStageEdges];
        bool ok[2 * kStageEdges];
#pragma unroll
        for (int j = 0; j < kStageEdges; ++j) {
            const int64_t i = t0 + t + (int64_t)j * kStageThreads;
            bool val = false;
            int32_t a = 0, c = 0;
            if (i < end) {
                a = u[i];
                c = v[i];
                val = (uint32_t)a < (uint32_t)n && (uint32_t)c < (uint32_t)n;
            }
            ok[2 * j] = ok[2 * j + 1] = val;
            p[2 * j] = make_int2(a, c);
            p[2 * j + 1] = make_int2(c, a);
            if (val) {
                rank[2 * j] = atomicAdd(&toff[a >> kShift], 1u);
                rank[2 * j + 1] = atomicAdd(&toff[c >> kShift], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the tile's bucket counts (B <= 2 * 1024 entries)
        {
            const uint32_t c0 = 2 * t < B ? toff[2 * t] : 0u;
            const uint32_t c1 = 2 * t + 1 < B ? toff[2 * t + 1] : 0u;
            const uint32_t s = c0 + c1;
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
                toff[B] = acc;
            }
            __syncthreads();
            const uint32_t ex = wsum[t >> 6] + incl - s;
            if (2 * t < B) toff[2 * t] = ex;
            if (2 * t + 1 < B) toff[2 * t + 1] = ex + c0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2 * kStageEdges; ++j)
            if (ok[j]) stage[toff[p[j].x >> kShift] + rank[j]] = p[j];
        __syncthreads();
        // contiguous runs per bucket: staged slot i -> its bucket's next free slot
        const uint32_t total = toff[B];
        for (uint32_t i = t; i < total; i += kStageThreads) {
            const int2 q = stage[i];
            const int k = q.x >> kShift;
            pairs[row[k] + run[k] + (i - toff[k])] = q;
        }
        __syncthreads();
        for (int k = t; k < B; k += kStageThreads) run[k] += toff[k + 1] - toff[k];
        __syncthreads();
    }
}

// per-vertex histogram update shared by the bucket pass and the standalone kernel
struct HistLds {
    uint32_t hx[kExactBins];
    uint32_t h64[64];
    unsigned long long best[kBlockD / 64];
};

__device__ __forceinline__ void hist_vertex(HistLds& L, uint32_t d, int32_t x, int32_t* tail, int64_t tail_cap,
                                            unsigned long long* tail_count, unsigned long long& best) {
    if (d < (uint32_t)kExactBins) atomicAdd(&L.hx[d], 1u);
    else {
        unsigned long long slot = atomic_add_agent(tail_count, 1ull);
        if ((int64_t)slot < tail_cap) tail[slot] = (int32_t)d;
    }
    atomicAdd(&L.h64[log_bin(d)], 1u);
    unsigned long long key = ((unsigned long long)d << 32) | (unsigned long long)(~(uint32_t)x);
    best = key > best ? key : best;
}

__device__ __forceinline__ void hist_flush(HistLds& L, unsigned long long best, unsigned long long* hist64,
                                           unsigned long long* histx, unsigned long long* argmax_key, int nthreads) {
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(best, off);
        best = o > best ? o : best;
    }
    if (lane_id() == 0) L.best[threadIdx.x >> 6] = best;
    __syncthreads();
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
__global__ __launch_bounds__(kBlockD) void bucket_degree_kernel(
    const int2* __restrict__ pairs, const unsigned long long* __restrict__ base, int32_t n,
    int32_t* __restrict__ deg, int count_pairs, int want_hist, unsigned long long* __restrict__ hist64,
    unsigned long long* __restrict__ histx, int32_t* __restrict__ tail, int64_t tail_cap,
    unsigned long long* __restrict__ tail_count, unsigned long long* __restrict__ argmax_key, int want_csr,
    int64_t* __restrict__ off, int32_t* __restrict__ adj) {
    __shared__ uint32_t cnt[kBsz];
    __shared__ HistLds L;
    __shared__ uint32_t wsum[kBlockD / 64];
    const int k = blockIdx.x;
    const int32_t x0 = k << kShift;
    int32_t nv = n - x0;
    if (nv > kBsz) nv = kBsz;
    for (int j = threadIdx.x; j < kBsz; j += kBlockD) cnt[j] = 0;
    for (int j = threadIdx.x; j < kExactBins; j += kBlockD) L.hx[j] = 0;
    if (threadIdx.x < 64) L.h64[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long beg = base[k], end = base[k + 1];
    if (!count_pairs) {
        // degrees already known (an earlier pass): only the CSR is built
        for (int j = threadIdx.x; j < nv; j += kBlockD) cnt[j] = (uint32_t)deg[x0 + j];
    }
    // every lane runs the same trip count so the wave-level aggregation can ballot
    for (unsigned long long i0 = beg; count_pairs && i0 < end; i0 += kBlockD) {
        const unsigned long long i = i0 + threadIdx.x;
        bool ok = i < end;
        int32_t x = ok ? pairs[i].x - x0 : -1;
        // aggregate lanes that hit the wave's first key (hub vertices)
        int32_t lead = __shfl(x, __builtin_ctzll(ballot(ok) | (1ull << 63)) & 63);
        uint64_t same = ballot(ok && x == lead);
        if (ok && x == lead) {
            if (lanes_below(same) == 0) atomicAdd(&cnt[lead], (uint32_t)__popcll(same));
        } else if (ok) {
            atomicAdd(&cnt[x], 1u);
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
    if (want_hist && count_pairs) hist_flush(L, best, hist64, histx, argmax_key, kBlockD);
    if (!want_csr) return;
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
    __syncthreads();
    for (unsigned long long i0 = beg; i0 < end; i0 += kBlockD) {
        const unsigned long long i = i0 + t;
        bool ok = i < end;
        int2 p = ok ? pairs[i] : make_int2(x0 - 1, 0);
        int32_t x = p.x - x0;
        // lanes sharing the wave's first key reserve their slots with one atomic
        int first = __builtin_ctzll(ballot(ok) | (1ull << 63)) & 63;
        int32_t lead = __shfl(x, first);
        uint64_t same = ballot(ok && x == lead);
        uint32_t rank = lanes_below(same);
        uint32_t basepos = 0;
        if (ok && x == lead && rank == 0) basepos = atomicAdd(&cnt[lead], (uint32_t)__popcll(same));
        int leader = __builtin_ctzll(same | (1ull << 63)) & 63;
        basepos = __shfl(basepos, leader);
        if (ok) {
            uint32_t pos = (x == lead) ? basepos + rank : atomicAdd(&cnt[x], 1u);
            adj[beg + pos] = p.y;
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
    for (int j = threadIdx.x; j < kExactBins; j += kBlockD) L.hx[j] = 0;
    if (threadIdx.x < 64) L.h64[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long best = 0;
    for (int64_t x = (int64_t)blockIdx.x * kBlockD + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlockD)
        hist_vertex(L, (uint32_t)deg[x], (int32_t)x, tail, tail_cap, tail_count, best);
    __syncthreads();
    hist_flush(L, best, hist64, histx, argmax_key, kBlockD);
}

// ------------------------------------------------------------------ host
int bucket_plan(int32_t n, int64_t m, BucketPlan* p) {
    p->B = (int32_t)(((int64_t)n + kBsz - 1) >> kShift);
    if (p->B < 1) p->B = 1;
    if (p->B > kMaxBuckets) return -1;
    int64_t nblk = (m + 65535) / 65536;   // ~64K edges per block chunk
    if (nblk < 1) nblk = 1;
    // the direct scatter (many buckets) keeps fewer blocks so the open output
    // runs stay within L2 and get written back as whole lines
    const int64_t maxblk = p->B > kStagedMaxB ? 256 : 1024;
    if (nblk > maxblk) nblk = maxblk;
    p->nblk = (int32_t)nblk;
    p->chunk = (m + nblk - 1) / nblk;
    if (p->chunk < 1) p->chunk = 1;
    return 0;
}

hipError_t launch_bucket_csr_from_deg(int32_t n, const BucketPlan& p, const BucketBufs& w, int32_t* deg,
                                      int64_t* off, int32_t* adj, hipStream_t s) {
    bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(w.pairs, w.base, n, deg, 0, 0, nullptr, nullptr, nullptr, 0,
                                                  nullptr, nullptr, 1, off, adj);
    return hipGetLastError();
}

hipError_t launch_bucket_degree(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const BucketPlan& p,
                                const BucketBufs& w, int32_t* deg, int want_hist, unsigned long long* hist64,
                                unsigned long long* histx, int32_t* tail, int64_t tail_cap,
                                unsigned long long* tail_count, unsigned long long* argmax_key, int want_csr,
                                int64_t* off, int32_t* adj, hipStream_t s) {
    const size_t lds = (size_t)p.B * sizeof(uint32_t);
    bucket_count_kernel<<<p.nblk, kBlock, lds, s>>>(u, v, m, n, p.chunk, p.B, w.counts, w.err);
    bucket_totals_kernel<<<(p.B + kBlock - 1) / kBlock, kBlock, 0, s>>>(w.counts, p.nblk, p.B, w.tot);
    bucket_scan_kernel<<<1, 1024, 0, s>>>(w.tot, p.B, w.base);
    bucket_offsets_kernel<<<(p.B + kBlock - 1) / kBlock, kBlock, 0, s>>>(w.counts, p.nblk, p.B, w.base, w.offs);
    if (p.B <= kStagedMaxB)
        bucket_scatter_staged_kernel<<<p.nblk, kStageThreads, 0, s>>>(u, v, m, n, p.chunk, p.B, w.offs, w.pairs);
    else
        bucket_scatter_kernel<<<p.nblk, kBlock, lds, s>>>(u, v, m, n, p.chunk, p.B, w.offs, w.pairs);
    bucket_degree_kernel<<<p.B, kBlockD, 0, s>>>(w.pairs, w.base, n, deg, 1, want_hist, hist64, histx, tail,
                                                  tail_cap, tail_count, argmax_key, want_csr, off, adj);
    return hipGetLastError();
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
