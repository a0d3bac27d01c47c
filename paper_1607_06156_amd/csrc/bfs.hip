// BFS step of Algorithm 2 (Section III-B): a direction-optimising BFS from one
// seed over the CSR, then the component label and the edge filter.
//
// The paper runs CombBLAS's distributed BFS on the relabelled graph; on one GPU
// the traversal switches between
//  * top-down levels: one thread per adjacency entry of the frontier queue
//    (edge-balanced, so a hub seed spreads over the whole grid); a neighbour is
//    claimed with atomicOr on the visited bitmap and appended to the next queue;
//  * bottom-up levels (Beamer, Asanovic & Patterson, SC 2012): every unvisited
//    vertex scans its neighbours until one lies in the frontier bitmap.  Each
//    workgroup owns a run of bitmap words, stages its visited and next-frontier
//    words in LDS, and writes them back once, so no global atomic touches the
//    bitmaps.
// The switch follows Beamer's rule: go bottom-up when the frontier's edges
// exceed 1/alpha of the unexplored edges (alpha = 14); return top-down when the
// frontier shrinks below n/beta vertices (beta = 24).
#include "bfs.hpp"
#include "common.hpp"

namespace ccmi {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ bool test_bit(const uint32_t* bits, int32_t x) {
    return (bits[x >> 5] >> (x & 31)) & 1u;
}

// ------------------------------------------------------ frontier degree scan
// pre[i] = sum_{j < i} deg(q[j]) within blocks of kScanB, bsum[b] = block total
constexpr int kScanB = 1024;

__global__ __launch_bounds__(kScanB) void qdeg_scan1_kernel(const int32_t* __restrict__ q, int64_t qn,
                                                            const int64_t* __restrict__ off,
                                                            int64_t* __restrict__ pre, int64_t* __restrict__ bsum) {
    __shared__ int64_t ws[kScanB / 64];
    int64_t i = (int64_t)blockIdx.x * kScanB + threadIdx.x;
    int64_t d = 0;
    if (i < qn) {
        int32_t x = q[i];
        d = off[x + 1] - off[x];
    }
    int64_t incl = d;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(incl, o);
        if (lane_id() >= o) incl += y;
    }
    if (lane_id() == 63) ws[threadIdx.x >> 6] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int w = 0; w < kScanB / 64; ++w) { int64_t t = ws[w]; ws[w] = acc; acc += t; }
        bsum[blockIdx.x] = acc;
    }
    __syncthreads();
    if (i < qn) pre[i] = ws[threadIdx.x >> 6] + incl - d;
}

// one block: exclusive scan of bsum[nb]; writes total to *total
__global__ __launch_bounds__(1024) void scan_small_i64_kernel(int64_t* __restrict__ a, int64_t nb,
                                                              int64_t* __restrict__ total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    int64_t s = 0;
    for (int64_t j = 0; j < per; ++j) {
        int64_t k = t * per + j;
        if (k < nb) s += a[k];
    }
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t x = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int64_t run = t ? part[t - 1] : 0;
    for (int64_t j = 0; j < per; ++j) {
        int64_t k = t * per + j;
        if (k < nb) {
            int64_t x = a[k];
            a[k] = run;
            run += x;
        }
    }
    if (t == 1023) *total = part[1023];
}

__global__ __launch_bounds__(kScanB) void qdeg_scan3_kernel(int64_t* __restrict__ pre, int64_t qn,
                                                            const int64_t* __restrict__ bsum,
                                                            const int64_t* __restrict__ total) {
    int64_t i = (int64_t)blockIdx.x * kScanB + threadIdx.x;
    if (i < qn) pre[i] += bsum[blockIdx.x];
    if (i == 0) pre[qn] = *total;
}

// ---------------------------------------------------------- top-down level
// One thread per adjacency entry of the frontier.  New vertices go to the
// next queue (one global atomic per block) and their degrees to ctr[1].
__global__ __launch_bounds__(kBlock) void topdown_kernel(const int32_t* __restrict__ q, int64_t qn,
                                                         const int64_t* __restrict__ pre,
                                                         const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ adj, uint32_t* vis,
                                                         int32_t* __restrict__ nq,
                                                         unsigned long long* __restrict__ ctr, int64_t per_block) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ unsigned long long qbase;
    const int64_t total = pre[qn];
    const int64_t e0 = (int64_t)blockIdx.x * per_block;
    int64_t e1 = e0 + per_block;
    if (e1 > total) e1 = total;
    unsigned long long mdeg = 0;
    for (int64_t eb = e0; eb < e1; eb += kBlock) {
        const int64_t e = eb + threadIdx.x;
        bool fresh = false;
        int32_t y = 0;
        if (e < e1) {
            // frontier index: last i with pre[i] <= e
            int64_t lo = 0, hi = qn - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= e) lo = mid; else hi = mid - 1;
            }
            int32_t x = q[lo];
            y = adj[off[x] + (e - pre[lo])];
            uint32_t bit = 1u << (y & 31);
            if (!(vis[y >> 5] & bit)) {
                uint32_t old = atomic_or_agent(&vis[y >> 5], bit);
                fresh = !(old & bit);
            }
            if (fresh) mdeg += (unsigned long long)(off[y + 1] - off[y]);
        }
        uint64_t mk = ballot(fresh);
        uint32_t tot;
        uint32_t woff = block_wave_offset((uint32_t)__popcll(mk), lds, &tot);
        if (tot) {
            if (threadIdx.x == 0) qbase = atomic_add_agent(&ctr[0], tot);
            __syncthreads();
            if (fresh) nq[qbase + woff + lanes_below(mk)] = y;
            __syncthreads();
        }
    }
    for (int o = 32; o > 0; o >>= 1) mdeg += __shfl_xor(mdeg, o);
    if (lane_id() == 0 && mdeg) atomic_add_agent(&ctr[1], mdeg);
}

// ----------------------------------------------- small levels in one workgroup
// A level whose frontier has few adjacency entries is microseconds of work,
// while a launch and a host round trip per level cost about 50 us (C1's 27
// levels took 1.4 ms that way).  One workgroup therefore runs consecutive
// top-down levels with workgroup barriers between them, from the frontier in
// q (qn vertices, their bits already set in vis), and stops before a level
// whose frontier has more than max_entries entries (the multi-launch levels
// take it), after max_levels levels, or when the frontier is empty.
//
// Per level: the frontier's degrees are scanned into a prefix, then each
// thread expands a contiguous share of the entries (a binary search for its
// first vertex, then a forward walk, four entries' reads in flight at a
// time) and appends new vertices to the other queue through an LDS counter.
// A frontier of at most kFewLds vertices lives in LDS as (row start, degree
// -> prefix), filled when its vertices are discovered (their offsets are read
// then anyway), so its scan, search and walk touch no global memory; larger
// frontiers use the global prefix array pre[].  The frontier it stops at is
// left in qa (vertex ids).
// out: [0] levels expanded, [1] vertices visited, [2] entries examined,
// [3] degree sum of the vertices visited, [4] vertices of the frontier left,
// [5] their degree sum.
constexpr int kFewThreads = 1024;
constexpr int kFewLds = 4096;
__global__ __launch_bounds__(kFewThreads) void bfs_few_kernel(const int64_t* __restrict__ off,
                                                              const int32_t* __restrict__ adj, int32_t* qa,
                                                              int32_t* qb, int64_t qn0, int64_t max_entries,
                                                              int32_t max_levels, uint32_t* vis, int64_t* pre,
                                                              unsigned long long* __restrict__ out) {
    __shared__ uint32_t s_pre[2][kFewLds + 1];   // degrees, then their exclusive prefix (entries <= 2^31)
    __shared__ int64_t s_row[2][kFewLds];        // row start of each frontier vertex
    __shared__ uint32_t s_found;
    __shared__ int64_t s_wsum[kFewThreads / 64];
    __shared__ int64_t s_carry;
    __shared__ unsigned long long s_fdeg;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    int32_t* q = qa;
    int32_t* nq = qb;
    int64_t qn = qn0, visited = 0, examined = 0;
    unsigned long long fdeg_all = 0;
    int32_t levels = 0;
    int64_t total = 0;
    int cb = 0;            // LDS buffer of the current frontier
    bool inl = false;      // the current frontier's degrees and rows are in s_pre[cb] / s_row[cb]
    for (;;) {
        // ---- exclusive scan of the frontier's degrees
        const bool lds = qn <= kFewLds;
        if (tid == 0) s_carry = 0;
        __syncthreads();
        for (int64_t r0 = 0; r0 < qn; r0 += kFewThreads) {
            const int64_t i = r0 + tid;
            int64_t d = 0;
            if (i < qn) {
                if (inl) {
                    d = s_pre[cb][i];
                } else {
                    const int32_t x = q[i];
                    const int64_t o0 = off[x];
                    d = off[x + 1] - o0;
                    if (lds) s_row[cb][i] = o0;
                }
            }
            int64_t x = d;
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) s_wsum[w] = x;
            __syncthreads();
            int64_t before = s_carry;
            for (int k = 0; k < w; ++k) before += s_wsum[k];
            if (i < qn) {
                if (lds) s_pre[cb][i] = (uint32_t)(before + x - d);
                else pre[i] = before + x - d;
            }
            __syncthreads();
            if (tid == 0) {
                int64_t t = 0;
                for (int k = 0; k < kFewThreads / 64; ++k) t += s_wsum[k];
                s_carry += t;
            }
            __syncthreads();
        }
        total = s_carry;
        if (qn == 0 || total > max_entries || levels >= max_levels) break;   // uniform: every thread read it
        if (tid == 0) {
            if (lds) s_pre[cb][qn] = (uint32_t)total;
            else pre[qn] = total;
            s_found = 0;
            s_fdeg = 0;
        }
        __syncthreads();
        // ---- expansion: thread tid takes entries [e0, e1)
        const int nb = cb ^ 1;
        const int64_t e0 = total * tid / kFewThreads, e1 = total * (tid + 1) / kFewThreads;
        auto P = [&](int64_t i) -> int64_t { return lds ? (int64_t)s_pre[cb][i] : pre[i]; };
        auto R = [&](int64_t i) -> int64_t { return lds ? s_row[cb][i] : off[q[i]]; };
        unsigned long long fdeg = 0;
        if (e0 < e1) {
            int64_t lo = 0, hi = qn - 1;   // last i with prefix <= e0
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (P(mid) <= e0) lo = mid; else hi = mid - 1;
            }
            int64_t i = lo, next = P(i + 1), base = R(i) - P(i);
            // eight entries per step, in three rounds of memory accesses:
            // their neighbours, the neighbours' bitmap words, then the
            // claiming atomics together with the candidates' row offsets
            constexpr int kG = 8;
            for (int64_t e = e0; e < e1; e += kG) {
                int32_t y[kG];
                bool ok[kG];
#pragma unroll
                for (int k = 0; k < kG; ++k) {
                    ok[k] = e + k < e1;
                    y[k] = 0;
                    if (ok[k]) {
                        while (e + k >= next) {
                            ++i;
                            next = P(i + 1);
                            base = R(i) - P(i);
                        }
                        y[k] = adj[base + e + k];
                    }
                }
                uint32_t wv[kG];
#pragma unroll
                for (int k = 0; k < kG; ++k) wv[k] = ok[k] ? vis[y[k] >> 5] : ~0u;
                bool cand[kG];
                uint32_t old[kG];
                int64_t o0[kG], o1[kG];
#pragma unroll
                for (int k = 0; k < kG; ++k) {
                    cand[k] = ok[k] && !(wv[k] & (1u << (y[k] & 31)));
                    old[k] = ~0u;
                    o0[k] = o1[k] = 0;
                    if (cand[k]) {
                        old[k] = atomic_or_agent(&vis[y[k] >> 5], 1u << (y[k] & 31));
                        o0[k] = off[y[k]];
                        o1[k] = off[y[k] + 1];
                    }
                }
#pragma unroll
                for (int k = 0; k < kG; ++k) {
                    if (!cand[k] || (old[k] & (1u << (y[k] & 31)))) continue;
                    const uint32_t slot = atomicAdd(&s_found, 1u);
                    nq[slot] = y[k];
                    const int64_t dy = o1[k] - o0[k];
                    fdeg += (unsigned long long)dy;
                    if (slot < (uint32_t)kFewLds) {
                        s_row[nb][slot] = o0[k];
                        s_pre[nb][slot] = (uint32_t)dy;
                    }
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) fdeg += __shfl_xor(fdeg, o);
        if (lane == 0 && fdeg) atomicAdd(&s_fdeg, fdeg);
        __syncthreads();
        qn = s_found;
        visited += qn;
        examined += total;
        fdeg_all += s_fdeg;
        ++levels;
        int32_t* t = q;
        q = nq;
        nq = t;
        inl = qn <= kFewLds;   // every new vertex's degree and row went to s_pre[nb] / s_row[nb]
        cb = nb;
        __syncthreads();   // every thread has read s_found and s_fdeg before the next level resets them
    }
    // the frontier left behind goes back to qa
    if (q != qa)
        for (int64_t i = tid; i < qn; i += kFewThreads) qa[i] = q[i];
    if (tid == 0) {
        out[0] = (unsigned long long)levels;
        out[1] = (unsigned long long)visited;
        out[2] = (unsigned long long)examined;
        out[3] = fdeg_all;
        out[4] = (unsigned long long)qn;
        out[5] = (unsigned long long)total;
    }
}

// --------------------------------------------------------- bottom-up level
// Grid-stride over runs of 8 bitmap words (256 vertices, one per thread).
__global__ __launch_bounds__(kBlock) void bottomup_kernel(int32_t n, const int64_t* __restrict__ off,
                                                          const int32_t* __restrict__ adj, uint32_t* __restrict__ vis,
                                                          const uint32_t* __restrict__ front,
                                                          uint32_t* __restrict__ next,
                                                          unsigned long long* __restrict__ ctr) {
    __shared__ uint32_t lvis[kBlock / 32];
    __shared__ uint32_t lnext[kBlock / 32];
    const int64_t words = ((int64_t)n + 31) >> 5;
    unsigned long long found = 0, mdeg = 0, exam = 0;
    for (int64_t w0 = (int64_t)blockIdx.x * (kBlock / 32); w0 < words; w0 += (int64_t)gridDim.x * (kBlock / 32)) {
        if (threadIdx.x < kBlock / 32) {
            int64_t w = w0 + threadIdx.x;
            lvis[threadIdx.x] = w < words ? vis[w] : 0xffffffffu;
            lnext[threadIdx.x] = 0;
        }
        __syncthreads();
        const int64_t x = w0 * 32 + threadIdx.x;
        const uint32_t bit = 1u << (threadIdx.x & 31);
        if (x < n && !(lvis[threadIdx.x >> 5] & bit)) {
            int64_t a = off[x], b = off[x + 1];
            for (int64_t j = a; j < b; ++j) {
                ++exam;
                int32_t y = adj[j];
                if (test_bit(front, y)) {
                    atomicOr(&lnext[threadIdx.x >> 5], bit);
                    ++found;
                    mdeg += (unsigned long long)(b - a);
                    break;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < kBlock / 32) {
            int64_t w = w0 + threadIdx.x;
            if (w < words) {
                next[w] = lnext[threadIdx.x];
                if (lnext[threadIdx.x]) vis[w] = lvis[threadIdx.x] | lnext[threadIdx.x];
            }
        }
        __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) {
        found += __shfl_xor(found, o);
        mdeg += __shfl_xor(mdeg, o);
        exam += __shfl_xor(exam, o);
    }
    __shared__ unsigned long long red[3][kWaves];
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = found;
        red[1][threadIdx.x >> 6] = mdeg;
        red[2][threadIdx.x >> 6] = exam;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long f = 0, d = 0, e = 0;
        for (int w = 0; w < kWaves; ++w) { f += red[0][w]; d += red[1][w]; e += red[2][w]; }
        if (f) atomic_add_agent(&ctr[0], f);
        if (d) atomic_add_agent(&ctr[1], d);
        if (e) atomic_add_agent(&ctr[2], e);
    }
}

// ------------------------------------------------------------ conversions
// queue -> bitmap (bits must be zero)
__global__ __launch_bounds__(kBlock) void queue_to_bits_kernel(const int32_t* __restrict__ q, int64_t qn,
                                                               uint32_t* bits) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < qn; i += (int64_t)gridDim.x * kBlock) {
        int32_t x = q[i];
        atomic_or_agent(&bits[x >> 5], 1u << (x & 31));
    }
}

// bitmap -> queue (order unspecified)
__global__ __launch_bounds__(kBlock) void bits_to_queue_kernel(const uint32_t* __restrict__ bits, int64_t words,
                                                               int32_t* __restrict__ q,
                                                               unsigned long long* __restrict__ qn) {
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ unsigned long long base;
    for (int64_t w0 = (int64_t)blockIdx.x * kBlock; w0 < words; w0 += (int64_t)gridDim.x * kBlock) {
        int64_t w = w0 + threadIdx.x;
        uint32_t word = w < words ? bits[w] : 0u;
        uint32_t c = (uint32_t)__popc(word);
        uint32_t incl = c;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(incl, o);
            if (lane_id() >= o) incl += y;
        }
        uint32_t tot;
        uint32_t woff = block_wave_offset(__shfl(incl, 63), lds, &tot);
        if (tot) {
            if (threadIdx.x == 0) base = atomic_add_agent(qn, tot);
            __syncthreads();
            uint32_t pos = (uint32_t)base + woff + incl - c;
            while (word) {
                int b = __builtin_ctz(word);
                q[(int64_t)pos++] = (int32_t)(w * 32 + b);
                word &= word - 1;
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------ label and filter
// *label = smallest visited id (int32 max if none)
__global__ __launch_bounds__(kBlock) void first_bit_kernel(const uint32_t* __restrict__ vis, int64_t words,
                                                           int32_t* __restrict__ label) {
    int32_t best = 0x7fffffff;
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < words; w += (int64_t)gridDim.x * kBlock) {
        uint32_t word = vis[w];
        if (word) {
            best = (int32_t)(w * 32 + __builtin_ctz(word));
            break;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        int32_t y = __shfl_xor(best, o);
        best = y < best ? y : best;
    }
    if (lane_id() == 0 && best != 0x7fffffff) atomic_min_agent(label, best);
}

// labels[x] = visited ? label : x
__global__ __launch_bounds__(kBlock) void bfs_label_kernel(const uint32_t* __restrict__ vis, int32_t n,
                                                           const int32_t* __restrict__ label,
                                                           int32_t* __restrict__ labels) {
    const int32_t c = *label;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += (int64_t)gridDim.x * kBlock)
        labels[x] = test_bit(vis, (int32_t)x) ? c : (int32_t)x;
}

// keep edge i iff its first endpoint is unvisited; block b handles the dense
// chunk [b*cap, (b+1)*cap) and writes survivors to segment b of out.
__global__ __launch_bounds__(kBlock) void filter_kernel(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                                        int64_t m, int32_t n, const uint32_t* __restrict__ vis,
                                                        SegList out, unsigned long long* __restrict__ bad) {
    __shared__ uint32_t lds[kWaves + 1];
    const int b = blockIdx.x;
    const int64_t base = (int64_t)b * out.cap;
    int64_t len = m - base;
    if (len > out.cap) len = out.cap;
    if (len < 0) len = 0;
    int2* dst = out.buf + base;
    uint32_t kept = 0, nbad = 0;
    constexpr int EPT = 4;
    for (int64_t t0 = 0; t0 < len; t0 += kBlock * EPT) {
        bool keep[EPT];
        int2 e[EPT];
        uint64_t mk[EPT];
        uint32_t pre[EPT], wk = 0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
            keep[k] = false;
            if (i < len) {
                int32_t a = u[base + i], c = v[base + i];
                e[k] = make_int2(a, c);
                if ((uint32_t)a >= (uint32_t)n || (uint32_t)c >= (uint32_t)n) ++nbad;
                else keep[k] = !test_bit(vis, a);
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            mk[k] = ballot(keep[k]);
            pre[k] = wk + lanes_below(mk[k]);
            wk += (uint32_t)__popcll(mk[k]);
        }
        uint32_t tot;
        uint32_t woff = block_wave_offset(wk, lds, &tot);
#pragma unroll
        for (int k = 0; k < EPT; ++k)
            if (keep[k]) dst[kept + woff + pre[k]] = e[k];
        kept += tot;
    }
    if (threadIdx.x == 0) out.count[b] = kept;
    for (int o = 32; o > 0; o >>= 1) nbad += __shfl_xor(nbad, o);
    if (lane_id() == 0 && nbad) atomic_add_agent(bad, nbad);
}

// CSR sanity: off[0] == 0, non-decreasing, off[n] == nadj, every adj entry in [0, n)
__global__ __launch_bounds__(kBlock) void csr_check_kernel(const int64_t* __restrict__ off, int32_t n,
                                                           const int32_t* __restrict__ adj, int64_t nadj,
                                                           unsigned long long* __restrict__ bad) {
    uint32_t nb = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n; i += stride) {
        int64_t o = off[i];
        if (i == 0 && o != 0) ++nb;
        if (i == n && o != nadj) ++nb;
        if (i < n && off[i + 1] < o) ++nb;
    }
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nadj; j += stride)
        if ((uint32_t)adj[j] >= (uint32_t)n) ++nb;
    for (int o = 32; o > 0; o >>= 1) nb += __shfl_xor(nb, o);
    if (lane_id() == 0 && nb) atomic_add_agent(bad, nb);
}

// sum of nseg counts -> *total
__global__ __launch_bounds__(kBlock) void sum_counts_kernel(const uint32_t* __restrict__ cnt, int32_t nseg,
                                                            unsigned long long* __restrict__ total) {
    __shared__ unsigned long long red[kWaves];
    unsigned long long s = 0;
    for (int i = threadIdx.x; i < nseg; i += kBlock) s += cnt[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0;
        for (int w = 0; w < kWaves; ++w) a += red[w];
        *total = a;
    }
}

// ------------------------------------------------------ rest from the CSR
// The edges a BFS leaves are those between unvisited vertices.  When the
// unvisited rows are short in total they are read from the CSR instead of
// probing the visited bitmap for every edge of the list: an edge lies in the
// rows of both of its ends and is taken from the row of its smaller end; a
// self-loop has two entries in its vertex's row and is taken once per pair.
// Each wave walks 64 consecutive vertices at a time: a row of up to
// kRestShort entries by its lane, a longer one by the whole wave.  COUNT:
// the number of edges per wave; else the edges, written as (smaller, larger)
// from the wave's offset (an exclusive prefix of the counts).
constexpr int kRestShort = 16;
constexpr int kRestV = 4096;   // vertices per block

__device__ __forceinline__ int64_t shfl_i64(int64_t x, int l) {
    const int32_t lo = __shfl((int32_t)(x & 0xffffffff), l);
    const int32_t hi = __shfl((int32_t)(x >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void rest_kernel(const uint32_t* __restrict__ vis, const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ adj, int32_t n,
                                                      int64_t* __restrict__ wcount, int32_t* __restrict__ fu,
                                                      int32_t* __restrict__ fv) {
    const int w = threadIdx.x >> 6, lane = lane_id();
    const int64_t gw = (int64_t)blockIdx.x * kWaves + w;
    const int64_t x0 = (int64_t)blockIdx.x * kRestV + (int64_t)w * (kRestV / kWaves);
    int64_t pos = COUNT ? 0 : wcount[gw];   // wave-uniform
    for (int step = 0; step < kRestV / kWaves / 64; ++step) {
        const int64_t xi = x0 + (int64_t)step * 64 + lane;
        const int32_t x = (int32_t)xi;
        const bool un = xi < n && !test_bit(vis, x);
        const int64_t o0 = un ? off[xi] : 0, o1 = un ? off[xi + 1] : 0;
        const bool shortrow = o1 - o0 <= kRestShort;
        // rows of up to kRestShort entries: this lane
        int32_t mine = 0, self = 0;
        if (shortrow)
            for (int64_t j = o0; j < o1; ++j) {
                const int32_t y = adj[j];
                mine += x < y;
                self += x == y;
            }
        mine += self >> 1;
        int32_t incl = mine;   // wave inclusive scan
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t t = __shfl_up(incl, d);
            if (lane >= d) incl += t;
        }
        const int32_t wtot = __shfl(incl, 63);
        if (!COUNT && mine > 0) {
            int64_t p = pos + incl - mine;
            for (int64_t j = o0; j < o1; ++j) {
                const int32_t y = adj[j];
                if (x < y) {
                    fu[p] = x;
                    fv[p] = y;
                    ++p;
                }
            }
            for (int32_t k = 0; k < (self >> 1); ++k, ++p) {
                fu[p] = x;
                fv[p] = x;
            }
        }
        pos += wtot;
        // longer rows: the whole wave walks each in turn
        uint64_t lm = ballot(!shortrow);
        while (lm) {
            const int l = __builtin_ctzll(lm);
            lm &= lm - 1;
            const int32_t xl = __shfl(x, l);
            const int64_t a0 = shfl_i64(o0, l), a1 = shfl_i64(o1, l);
            int64_t selfw = 0;
            for (int64_t j0 = a0; j0 < a1; j0 += 64) {
                const int64_t j = j0 + lane;
                const int32_t y = j < a1 ? adj[j] : -1;   // ids are >= 0: -1 matches nothing
                const uint64_t km = ballot(xl < y);
                selfw += __popcll(ballot(y == xl));
                if (!COUNT && xl < y) {
                    const int64_t p = pos + lanes_below(km);
                    fu[p] = xl;
                    fv[p] = y;
                }
                pos += __popcll(km);
            }
            const int64_t half = selfw >> 1;
            if (!COUNT)
                for (int64_t k = lane; k < half; k += 64) {
                    fu[pos + k] = xl;
                    fv[pos + k] = xl;
                }
            pos += half;
        }
    }
    if (COUNT && lane == 0) wcount[gw] = pos;
}

// segmented int2 list -> dense SoA (segment b starts at prefix[b])
__global__ __launch_bounds__(kBlock) void seg_to_soa_kernel(SegList in, const int64_t* __restrict__ prefix,
                                                            int32_t* __restrict__ fu, int32_t* __restrict__ fv) {
    const int b = blockIdx.x;
    const uint32_t c = in.count[b];
    const int2* src = in.buf + (int64_t)b * in.cap;
    const int64_t o = prefix[b];
    for (uint32_t j = threadIdx.x; j < c; j += kBlock) {
        int2 e = src[j];
        fu[o + j] = e.x;
        fv[o + j] = e.y;
    }
}

__global__ void counts_to_i64_kernel(const uint32_t* __restrict__ c, int64_t* __restrict__ o, int32_t k) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) o[i] = c[i];
}

// ------------------------------------------------------------------ host
static int grid_cap(int64_t work, int per, int cap) {
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_qdeg_scan(const int32_t* q, int64_t qn, const int64_t* off, int64_t* pre, int64_t* bsum,
                            int64_t* total, hipStream_t s) {
    int64_t nb = (qn + kScanB - 1) / kScanB;
    if (nb < 1) nb = 1;
    qdeg_scan1_kernel<<<(unsigned)nb, kScanB, 0, s>>>(q, qn, off, pre, bsum);
    scan_small_i64_kernel<<<1, 1024, 0, s>>>(bsum, nb, total);
    qdeg_scan3_kernel<<<(unsigned)nb, kScanB, 0, s>>>(pre, qn, bsum, total);
    return hipGetLastError();
}

hipError_t launch_topdown(const int32_t* q, int64_t qn, const int64_t* pre, int64_t total_entries,
                          const int64_t* off, const int32_t* adj, uint32_t* vis, int32_t* nq,
                          unsigned long long* ctr, hipStream_t s) {
    // ~4096 entries per block keeps the per-block queue atomics few
    int64_t per = 4096;
    int64_t g = (total_entries + per - 1) / per;
    if (g > 65535) {
        per = (total_entries + 65534) / 65535;
        per = (per + kBlock - 1) / kBlock * kBlock;
        g = (total_entries + per - 1) / per;
    }
    if (g < 1) g = 1;
    topdown_kernel<<<(unsigned)g, kBlock, 0, s>>>(q, qn, pre, off, adj, vis, nq, ctr, per);
    return hipGetLastError();
}

hipError_t launch_bfs_few(const int64_t* off, const int32_t* adj, int32_t* qa, int32_t* qb, int64_t qn,
                          int64_t max_entries, int32_t max_levels, uint32_t* vis, int64_t* pre,
                          unsigned long long* out, hipStream_t s) {
    if (qn < 0 || max_levels < 1) return hipErrorInvalidValue;
    bfs_few_kernel<<<1, kFewThreads, 0, s>>>(off, adj, qa, qb, qn, max_entries, max_levels, vis, pre, out);
    return hipGetLastError();
}

hipError_t launch_bottomup(int32_t n, const int64_t* off, const int32_t* adj, uint32_t* vis, const uint32_t* front,
                           uint32_t* next, unsigned long long* ctr, hipStream_t s) {
    int g = grid_cap(((int64_t)n + 255) / 256, 1, 2048);
    bottomup_kernel<<<g, kBlock, 0, s>>>(n, off, adj, vis, front, next, ctr);
    return hipGetLastError();
}

hipError_t launch_queue_to_bits(const int32_t* q, int64_t qn, uint32_t* bits, hipStream_t s) {
    if (qn <= 0) return hipSuccess;
    queue_to_bits_kernel<<<grid_cap(qn, kBlock, 4096), kBlock, 0, s>>>(q, qn, bits);
    return hipGetLastError();
}

hipError_t launch_bits_to_queue(const uint32_t* bits, int64_t words, int32_t* q, unsigned long long* qn,
                                hipStream_t s) {
    bits_to_queue_kernel<<<grid_cap(words, kBlock, 1024), kBlock, 0, s>>>(bits, words, q, qn);
    return hipGetLastError();
}


hipError_t launch_bfs_label(const uint32_t* vis, int32_t n, int32_t* label, int32_t* labels, hipStream_t s) {
    int64_t words = ((int64_t)n + 31) >> 5;
    first_bit_kernel<<<grid_cap(words, kBlock, 1024), kBlock, 0, s>>>(vis, words, label);
    bfs_label_kernel<<<grid_cap(n, kBlock * 4, 4096), kBlock, 0, s>>>(vis, n, label, labels);
    return hipGetLastError();
}

hipError_t launch_filter(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const uint32_t* vis, SegList out,
                         unsigned long long* total, unsigned long long* bad, hipStream_t s) {
    filter_kernel<<<out.nseg, kBlock, 0, s>>>(u, v, m, n, vis, out, bad);
    sum_counts_kernel<<<1, kBlock, 0, s>>>(out.count, out.nseg, total);
    return hipGetLastError();
}

int64_t rest_waves(int32_t n) { return ((int64_t)n + kRestV - 1) / kRestV * kWaves; }

hipError_t launch_rest_count(const uint32_t* vis, const int64_t* off, const int32_t* adj, int32_t n, int64_t* wcount,
                             int64_t* total, hipStream_t s) {
    const int64_t blocks = ((int64_t)n + kRestV - 1) / kRestV;
    if (blocks < 1) return hipSuccess;
    rest_kernel<true><<<(unsigned)blocks, kBlock, 0, s>>>(vis, off, adj, n, wcount, nullptr, nullptr);
    scan_small_i64_kernel<<<1, 1024, 0, s>>>(wcount, blocks * kWaves, total);
    return hipGetLastError();
}

hipError_t launch_rest_emit(const uint32_t* vis, const int64_t* off, const int32_t* adj, int32_t n,
                            const int64_t* woff, int32_t* fu, int32_t* fv, hipStream_t s) {
    const int64_t blocks = ((int64_t)n + kRestV - 1) / kRestV;
    if (blocks < 1) return hipSuccess;
    rest_kernel<false><<<(unsigned)blocks, kBlock, 0, s>>>(vis, off, adj, n, (int64_t*)woff, fu, fv);
    return hipGetLastError();
}

hipError_t launch_csr_check(const int64_t* off, int32_t n, const int32_t* adj, int64_t nadj,
                            unsigned long long* bad, hipStream_t s) {
    int64_t work = nadj > (int64_t)n + 1 ? nadj : (int64_t)n + 1;
    csr_check_kernel<<<grid_cap(work, kBlock * 8, 4096), kBlock, 0, s>>>(off, n, adj, nadj, bad);
    return hipGetLastError();
}

hipError_t launch_seg_to_soa(SegList in, int64_t* prefix_scratch, int64_t* total_scratch, int32_t* fu, int32_t* fv,
                             hipStream_t s) {
    counts_to_i64_kernel<<<grid_cap(in.nseg, kBlock, 64), kBlock, 0, s>>>(in.count, prefix_scratch, in.nseg);
    scan_small_i64_kernel<<<1, 1024, 0, s>>>(prefix_scratch, in.nseg, total_scratch);
    seg_to_soa_kernel<<<in.nseg, kBlock, 0, s>>>(in, prefix_scratch, fu, fv);
    return hipGetLastError();
}

}  // namespace ccmi
