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
#include "sv_device.hpp"

namespace ccmi {

__global__ __launch_bounds__(kBlock) void sv_init_kernel(int32_t* __restrict__ parent, int32_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) parent[i] = (int32_t)i;
}

// One pass: hook + compact over one block segment of edges.
// SOA: edges come from the caller's u[], v[] (dense); the block works on
// segment b = seg0 + blockIdx.x, edges [b*cap, min((b+1)*cap, m)), and checks
// ids against [0, n).  Else from segment b of `in`.
template <bool SOA>
__global__ __launch_bounds__(kBlock) void sv_pass_kernel(const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                                         int64_t m, int32_t n, int32_t seg0, SegList in,
                                                         int32_t* parent, SegList out, int write_out, int max_link,
                                                         int32_t* __restrict__ hooked,
                                                         uint32_t* __restrict__ hooked_count,
                                                         unsigned long long* __restrict__ totals) {
    __shared__ uint32_t lds[kWaves + 1];
    const int b = seg0 + blockIdx.x;
    int2* dst = out.buf + (int64_t)b * out.cap;
    int32_t* hdst = hooked + (int64_t)b * out.cap;
    uint32_t kept_off = 0, hook_off = 0, bad = 0, nlong = 0;
    if (SOA) {
        const int64_t base = (int64_t)b * out.cap;
        int64_t len = m - base;
        if (len > out.cap) len = out.cap;
        if (len < 0) len = 0;
        auto load = [&](int64_t i, int32_t* a, int32_t* c) -> bool {
            *a = u[base + i];
            *c = v[base + i];
            if ((uint32_t)*a >= (uint32_t)n || (uint32_t)*c >= (uint32_t)n) {
                ++bad;
                return false;
            }
            return true;
        };
        sv_segment(len, load, parent, dst, hdst, write_out != 0, max_link, kept_off, hook_off, nlong, lds);
    } else {
        const int2* src = in.buf + (int64_t)b * in.cap;
        const int64_t len = in.count[b];
        auto load = [&](int64_t i, int32_t* a, int32_t* c) -> bool {
            const int2 e = src[i];
            *a = e.x;
            *c = e.y;
            return true;
        };
        sv_segment(len, load, parent, dst, hdst, write_out != 0, max_link, kept_off, hook_off, nlong, lds);
    }
    // per-block results (no global atomics on the fast path)
    if (threadIdx.x == 0) {
        out.count[b] = kept_off;
        hooked_count[b] = hook_off;
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
// seg_lo .. nseg-1 only (the roots hooked after the last full flatten).
constexpr int kTotThreads = 1024;
__global__ __launch_bounds__(kTotThreads) void sv_totals_kernel(const uint32_t* __restrict__ hooked_count,
                                                                const uint32_t* __restrict__ kept_count, int32_t nseg,
                                                                int32_t seg_lo, unsigned long long* __restrict__ totals) {
    constexpr int W = kTotThreads / 64;
    __shared__ unsigned long long red[3][W];
    unsigned long long sk = 0, sh = 0, sf = 0;
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
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = sk;
        red[1][threadIdx.x >> 6] = sh;
        red[2][threadIdx.x >> 6] = sf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, c = 0, f = 0;
        for (int w = 0; w < W; ++w) { a += red[0][w]; c += red[1][w]; f += red[2][w]; }
        totals[0] = a;
        totals[1] = c;
        totals[3] = f;
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
__global__ __launch_bounds__(kBlock) void sv_finalize_kernel(int32_t* parent, int32_t n,
                                                             unsigned long long* open) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    bool left = false;
    for (; i < n; i += stride) {
        int32_t p = parent[i];
        if (p == (int32_t)i) continue;
        bool root;
        int32_t r = find_bounded(parent, p, &root);
        if (r != p) parent[i] = r;
        left |= !root;
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

hipError_t launch_sv_pass_soa(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* parent,
                              SegList out, int32_t seg0, int32_t nblocks, int write_out, int max_link,
                              int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals, hipStream_t s) {
    if (seg0 < 0 || nblocks < 1 || seg0 + nblocks > out.nseg) return hipErrorInvalidValue;
    SegList none{nullptr, 0, 0, nullptr};
    sv_pass_kernel<true><<<nblocks, kBlock, 0, s>>>(u, v, m, n, seg0, none, parent, out, write_out, max_link, hooked,
                                                    hooked_count, totals);
    return hipGetLastError();
}

hipError_t launch_sv_pass_seg(SegList in, int32_t seg0, int32_t nblocks, int32_t* parent, SegList out, int write_out,
                              int max_link, int32_t* hooked, uint32_t* hooked_count, unsigned long long* totals,
                              hipStream_t s) {
    if (seg0 < 0 || nblocks < 1 || seg0 + nblocks > in.nseg || in.nseg > out.nseg) return hipErrorInvalidValue;
    sv_pass_kernel<false><<<nblocks, kBlock, 0, s>>>(nullptr, nullptr, 0, 0, seg0, in, parent, out, write_out,
                                                     max_link, hooked, hooked_count, totals);
    return hipGetLastError();
}

hipError_t launch_sv_shortcut(int32_t* parent, const int32_t* hooked, const uint32_t* hooked_count, int64_t cap,
                              int32_t nseg, hipStream_t s) {
    sv_shortcut_kernel<<<nseg, kBlock, 0, s>>>(parent, hooked, hooked_count, cap);
    return hipGetLastError();
}

hipError_t launch_sv_totals(const uint32_t* hooked_count, const uint32_t* kept_count, int32_t nseg, int32_t seg_lo,
                            unsigned long long* totals, hipStream_t s) {
    sv_totals_kernel<<<1, kTotThreads, 0, s>>>(hooked_count, kept_count, nseg, seg_lo, totals);
    return hipGetLastError();
}

hipError_t launch_sv_finalize(int32_t* parent, int32_t n, unsigned long long* open, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    sv_finalize_kernel<<<grid_for(n, 4), kBlock, 0, s>>>(parent, n, open);
    return hipGetLastError();
}

}  // namespace ccmi
