// Batched labelling: G independent graphs in one persistent launch.
//
// Graph g's local ids are shifted by vert_off[g], which turns the batch into one
// graph on vert_off[G] vertices whose components never cross graphs.  The
// shift is monotone, so the minimum global id of a component is vert_off[g]
// plus its minimum local id: the canonical labels of Fig. 1(b) survive, and
// subtracting vert_off[g] at the end gives the graph-local labels.
//
// The whole SV iteration (Section III-A) runs inside one cooperative launch.
// The concatenated edge list is cut into tiles of 1024 edges; every tile keeps
// its own output segment (survivors of tile t go to slots [t*1024, ...)), so
// no global atomic places output.  Pass after pass each workgroup hooks and
// compacts its tiles and waits at a grid barrier.  After the barrier every
// workgroup sums the per-block survivor and hook partials and takes the same
// decisions (stop; pointer-jump the roots hooked in its tiles or leave them to
// the final compression), so convergence is decided on the device and the
// host waits once.  Small graphs finish in the first passes and
// simply drop out of the active tiles (Section III-A.4: completed work leaves
// the working set).
#include "batched.hpp"
#include "common.hpp"
#include "sv_device.hpp"

namespace ccmi {

struct BatchArgs {
    const int32_t* u;
    const int32_t* v;
    const int64_t* edge_off;
    const int64_t* vert_off;
    int32_t G;
    int64_t m;            // edge_off[G] (read by the host)
    int32_t n;            // vert_off[G]
    int32_t* parent;      // labels: global roots, then local labels
    int2* buf0;           // tile segments, ping-pong
    int2* buf1;
    uint32_t* cnt0;       // per-tile survivor counts (ping-pong)
    uint32_t* cnt1;
    uint32_t* hcnt;       // per-tile hooked counts
    int32_t* hooked;      // per-tile hooked roots
    unsigned int* bar;    // [0] arrivals, [1] generation
    unsigned long long* status;  // [0] error bits, [1] passes, [2] range errors, [4] labels left unshifted
    int32_t max_passes;
    int32_t max_link;     // hook attempts per edge per pass (see sv_segment)
    uint64_t barrier_ticks;     // spin limit of a grid barrier, in 100 MHz wall-clock ticks
    unsigned long long* part;   // per-block partials: survivors, hooks, finds stopped at the hop
                                // bound (2 x gridDim each)
    unsigned long long* bstat;  // per block, over all passes (gridDim each): atomics issued, walk
                                // reads, active edges read, survivors written
};

constexpr int64_t kTileE = (int64_t)kBlock * kEPT;   // edges (or vertices) per tile

enum : unsigned long long { kErrRange = 1, kErrOffsets = 2, kErrBarrier = 4, kErrPasses = 8 };
constexpr int kStampBase = 8;    // status[8 + i]: wall clock when barrier i was passed
// status[kDeep] = 1: the final compression left a root beyond the walk bound;
// the labels stay global and unflattened, and the host finishes them
constexpr int kDeep = 4;
constexpr unsigned long long kLazyJump = 8;   // jump hooked roots only if hooks <= 8 x survivors
constexpr int kMaxStamps = 40;

__device__ __forceinline__ void stamp(unsigned long long* status, int i) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && i < kMaxStamps) status[kStampBase + i] = wall_clock64();
}

__device__ __forceinline__ unsigned long long load_status(unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sense-reversing grid barrier for a co-resident (cooperative) grid.  The spin
// is bounded (by default ~5 s): past the limit it flags an error, and a flagged
// error releases every later barrier at once, so all workgroups always exit.
__device__ void grid_barrier(unsigned int* bar, unsigned long long* status, uint64_t limit) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // release this block's writes (agent scope)
        const unsigned int gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&bar[1], gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (load_status(status) & kErrBarrier) break;
                if (wall_clock64() - t0 > limit) {
                    __hip_atomic_fetch_or(&status[0], (unsigned long long)kErrBarrier, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();   // acquire
    }
    __syncthreads();
}

// graph of edge / vertex index i: first g with off[g+1] > i (off non-decreasing, off[G] > i)
__device__ __forceinline__ int32_t graph_of(const int64_t* off, int32_t G, int64_t i) {
    int32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (off[mid + 1] > i) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs (workgroup b runs on XCD b % 8).  The tiles are cut into 8 contiguous
// ranges, one per XCD, and the workgroups of one XCD walk their range in
// lock-step (tile j, j + nbx, ...), so the tiles an XCD processes at any
// moment are neighbours: they belong to one or a few graphs, whose parent
// ranges stay in that XCD's L2.
struct TileWalk {
    int64_t first, step, end;
    __device__ TileWalk(int64_t T, int b, int nb) {
        const int x = b & 7, j = b >> 3;
        const int nbx = nb >> 3;
        const int64_t Tx = (T + 7) / 8;
        first = (int64_t)x * Tx + j;
        step = nbx;
        end = (int64_t)(x + 1) * Tx;
        if (end > T) end = T;
    }
};

// At most 80 VGPRs, so that 6 waves per SIMD stay resident (the persistent
// grid is sized to what is co-resident); 7 would spill.
__global__ __launch_bounds__(kBlock, 6) void batched_kernel(BatchArgs A) {
    __shared__ uint32_t lds[kWaves + 1];
    // sh_total / sh_hooks / sh_long: grid-wide sums, written and read only at
    // the top of a pass; sh_blong: this workgroup's count of finds stopped at
    // the hop bound, summed at the end of a pass and read by thread 0 only
    __shared__ unsigned long long sh_total, sh_hooks, sh_long, sh_blong;
    __shared__ int32_t sh_g;
    const int b = blockIdx.x;
    const int nb = gridDim.x;
    const int64_t gstride = (int64_t)nb * kBlock;
    const int64_t gtid = (int64_t)b * kBlock + threadIdx.x;
    const int64_t T = (A.m + kTileE - 1) / kTileE;           // edge tiles
    if (nb < 8 || (nb & 7)) {                                 // the tile walk needs 8 | grid
        if (b == 0 && threadIdx.x == 0)
            __hip_atomic_fetch_or(&A.status[0], (unsigned long long)kErrOffsets, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    const TileWalk tw(T, b, nb);
    const int64_t TV = ((int64_t)A.n + kTileE - 1) / kTileE;   // vertex tiles

    // ---- init: identity forest, offset checks
    for (int64_t x = gtid; x < A.n; x += gstride) A.parent[x] = (int32_t)x;
    for (int64_t g = gtid; g < A.G; g += gstride) {
        if (A.edge_off[g + 1] < A.edge_off[g] || A.vert_off[g + 1] < A.vert_off[g])
            __hip_atomic_fetch_or(&A.status[0], (unsigned long long)kErrOffsets, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_barrier(A.bar, A.status, A.barrier_ticks);
    if (load_status(A.status)) return;
    stamp(A.status, 0);

    // ---- pass 0, straight from the caller's SoA list.  Thread 0 finds each
    // tile's first graph (one binary search); every thread then walks forward
    // to the graphs of its own edges (it sees them in increasing order),
    // shifts the ids to global ones and drops (and counts) edges with an id
    // outside their graph.
    uint32_t bad = 0, nlong = 0;
    uint32_t natom = 0, nchase = 0;   // per thread, over all passes
    unsigned long long block_kept = 0, block_hooks = 0;
    unsigned long long tot_read = 0, tot_kept = 0;   // this block, over all passes (thread 0's count)
    int32_t tg = -1;   // thread 0: graph of the last tile's first edge
    for (int64_t t = tw.first; t < tw.end; t += tw.step) {
        const int64_t e0 = t * kTileE;
        int64_t len = A.m - e0;
        if (len > kTileE) len = kTileE;
        __syncthreads();   // every thread has read the previous tile's sh_g
        if (threadIdx.x == 0) {
            // this block's tiles come in increasing order: from the last
            // tile's graph, walk forward (one binary search for the first)
            if (tg < 0) tg = graph_of(A.edge_off, A.G, e0);
            else
                while (A.edge_off[tg + 1] <= e0) ++tg;
            sh_g = tg;
        }
        __syncthreads();
        int32_t g = sh_g;
        // All of the thread's edge reads go out first (non-temporal: the
        // list is read once); its edges arrive in increasing order, so g only
        // walks forward.  Indices past the tile's end read its first edge.
        auto loader = [&](int64_t t0, int32_t* a, int32_t* c, bool* valid) {
            int64_t e[kEPT];
            bool in[kEPT];
            int32_t x[kEPT], y[kEPT];
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                const int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
                in[k] = i < len;
                e[k] = e0 + (in[k] ? i : 0);
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                x[k] = __builtin_nontemporal_load(A.u + e[k]);
                y[k] = __builtin_nontemporal_load(A.v + e[k]);
            }
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                valid[k] = false;
                if (!in[k]) continue;
                while (A.edge_off[g + 1] <= e[k]) ++g;
                const int64_t v0 = A.vert_off[g];
                const int64_t nl = A.vert_off[g + 1] - v0;
                if (x[k] < 0 || y[k] < 0 || (int64_t)x[k] >= nl || (int64_t)y[k] >= nl) {
                    ++bad;
                    continue;
                }
                a[k] = (int32_t)(v0 + x[k]);
                c[k] = (int32_t)(v0 + y[k]);
                valid[k] = true;
            }
        };
        uint32_t kept = 0, hk = 0;
        if (len > 0)
            sv_segment(len, loader, A.parent, A.buf0 + t * kTileE, A.hooked + t * kTileE, true, A.max_link, kept, hk,
                       nlong, lds, natom, nchase);
        if (threadIdx.x == 0) {
            A.cnt0[t] = kept;
            A.hcnt[t] = hk;
        }
        block_kept += kept;
        block_hooks += hk;
        tot_read += len > 0 ? (unsigned long long)len : 0ull;
    }
    tot_kept += block_kept;
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o);
    if (lane_id() == 0 && bad) {
        __hip_atomic_fetch_add(&A.status[2], (unsigned long long)bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(&A.status[0], (unsigned long long)kErrRange, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long* const part_base = A.part;
    unsigned long long* part_rd = part_base;
    for (int o = 32; o > 0; o >>= 1) nlong += __shfl_xor(nlong, o);
    if (threadIdx.x == 0) sh_blong = 0;
    __syncthreads();
    if (lane_id() == 0 && nlong) atomicAdd(&sh_blong, (unsigned long long)nlong);
    __syncthreads();
    if (threadIdx.x == 0) {
        part_base[b] = block_kept;
        part_base[2 * nb + b] = block_hooks;
        part_base[4 * nb + b] = sh_blong;
    }

    int pass = 1;
    int2* in = A.buf0;
    int2* out = A.buf1;
    uint32_t* cin = A.cnt0;
    uint32_t* cout = A.cnt1;
    for (;;) {
        grid_barrier(A.bar, A.status, A.barrier_ticks);
        if (load_status(A.status)) return;
        stamp(A.status, pass);
        // every block sums the same partials and takes the same decisions
        unsigned long long s = 0, sh = 0, sl = 0;
        for (int i = threadIdx.x; i < nb; i += kBlock) {
            s += part_rd[i];
            sh += part_rd[2 * nb + i];
            sl += part_rd[4 * nb + i];
        }
        for (int o = 32; o > 0; o >>= 1) {
            s += __shfl_xor(s, o);
            sh += __shfl_xor(sh, o);
            sl += __shfl_xor(sl, o);
        }
        if (threadIdx.x == 0) {
            sh_total = 0;
            sh_hooks = 0;
            sh_long = 0;
        }
        __syncthreads();
        if (lane_id() == 0) {
            atomicAdd(&sh_total, s);
            atomicAdd(&sh_hooks, sh);
            atomicAdd(&sh_long, sl);
        }
        __syncthreads();
        const unsigned long long total = sh_total, hooks = sh_hooks, deep = sh_long;
        if (total == 0) break;   // the final compression resolves every link
        // Pointer jumping of the roots hooked in this block's tiles, unless
        // they far outnumber the surviving edges (typically after the first
        // pass, when nearly every vertex was hooked): then the next pass's
        // finds walk the extra links of the few survivors instead, and the
        // final compression flattens everything once.  The jumped roots were
        // hooked before the barrier, so they are no longer roots, and a hook
        // of the next pass only ever lands on a root: the next pass may start
        // beside these plain stores.
        //
        // If some find of the pass stopped at the hop bound, every vertex of
        // this block's tiles is moved up instead (at most kMaxHops links), so
        // deep chains shrink by that factor per pass.  That sweep cannot tell
        // a vertex linked before the barrier from a root that another
        // workgroup's next pass has just hooked; a plain store to such a
        // vertex could erase a second hook's atomicMin and lose a connection.
        // So the sweep ends at a grid barrier of its own before any hook of
        // the next pass.
        if (deep > 0) {
            const TileWalk vw(TV, b, nb);
            for (int64_t t = vw.first; t < vw.end; t += vw.step) {
                for (int64_t x = t * kTileE + threadIdx.x; x < (t + 1) * kTileE && x < A.n; x += kBlock) {
                    const int32_t p = A.parent[x];
                    bool root;
                    if (p != (int32_t)x) A.parent[x] = find_bounded(A.parent, p, &root);
                }
            }
            grid_barrier(A.bar, A.status, A.barrier_ticks);
            if (load_status(A.status)) return;
        } else if (hooks <= kLazyJump * total) {
            for (int64_t t = tw.first; t < tw.end; t += tw.step) {
                const uint32_t hc = A.hcnt[t];
                const int32_t* h = A.hooked + t * kTileE;
                for (uint32_t j = threadIdx.x; j < hc; j += kBlock) {
                    const int32_t x = h[j];
                    bool root;
                    A.parent[x] = find_bounded(A.parent, x, &root);
                }
            }
        }
        if (A.max_passes > 0 && pass >= A.max_passes) {
            if (b == 0 && threadIdx.x == 0)
                __hip_atomic_fetch_or(&A.status[0], (unsigned long long)kErrPasses, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        // Partials alternate between two arrays: other blocks may still be
        // summing the previous pass's array while this block writes, and an
        // array is written again only after every block has passed the next
        // barrier, i.e. finished summing it.
        unsigned long long* part_out = part_base + (pass & 1) * nb;
        block_kept = 0;
        block_hooks = 0;
        nlong = 0;
        for (int64_t t = tw.first; t < tw.end; t += tw.step) {
            const uint32_t len = cin[t];
            uint32_t kept = 0, hk = 0;
            if (len) {
                const int2* src = in + t * kTileE;
                auto loader = [&](int64_t t0, int32_t* a, int32_t* c, bool* valid) {
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        const int64_t i = t0 + threadIdx.x + (int64_t)k * kBlock;
                        valid[k] = i < (int64_t)len;
                        const int2 e = src[valid[k] ? i : 0];
                        a[k] = e.x;
                        c[k] = e.y;
                    }
                };
                sv_segment((int64_t)len, loader, A.parent, out + t * kTileE, A.hooked + t * kTileE, true, A.max_link,
                           kept, hk, nlong, lds, natom, nchase);
            }
            if (threadIdx.x == 0) {
                cout[t] = kept;
                A.hcnt[t] = hk;
            }
            block_kept += kept;
            block_hooks += hk;
            tot_read += len;
        }
        tot_kept += block_kept;
        for (int o = 32; o > 0; o >>= 1) nlong += __shfl_xor(nlong, o);
        if (threadIdx.x == 0) sh_blong = 0;
        __syncthreads();
        if (lane_id() == 0 && nlong) atomicAdd(&sh_blong, (unsigned long long)nlong);
        __syncthreads();
        if (threadIdx.x == 0) {
            part_out[b] = block_kept;
            part_out[2 * nb + b] = block_hooks;
            part_out[4 * nb + b] = sh_blong;
        }
        part_rd = part_out;
        ++pass;
        int2* tt = in; in = out; out = tt;
        uint32_t* tc = cin; cin = cout; cout = tc;
    }
    if (b == 0 && threadIdx.x == 0) A.status[1] = (unsigned long long)pass;
    // this block's counts for the byte model (sh_total / sh_hooks are free:
    // every thread has read them before the loop ended)
    __syncthreads();
    {
        unsigned long long sa = natom, sc = nchase;
        for (int o = 32; o > 0; o >>= 1) {
            sa += __shfl_xor(sa, o);
            sc += __shfl_xor(sc, o);
        }
        if (threadIdx.x == 0) {
            sh_total = 0;
            sh_hooks = 0;
        }
        __syncthreads();
        if (lane_id() == 0) {
            atomicAdd(&sh_total, sa);
            atomicAdd(&sh_hooks, sc);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            A.bstat[b] = sh_total;
            A.bstat[nb + b] = sh_hooks;
            A.bstat[2 * nb + b] = tot_read;
            A.bstat[3 * nb + b] = tot_kept;
        }
    }

    // ---- final labels: compress to roots, then shift to graph-local ids.
    // A root beyond the walk bound (a chain deeper than kMaxHops links) leaves
    // the labels global; the host then finishes the flatten and the shift.
    const TileWalk vw(TV, b, nb);
    bool left = false;
    // a tile's kTileE / kBlock vertices per thread walk up in lock-step, so
    // their dependent reads overlap
    constexpr int kV = (int)(kTileE / kBlock);
    for (int64_t t = vw.first; t < vw.end; t += vw.step) {
        int32_t x[kV], p[kV], q[kV];
        bool act[kV];
#pragma unroll
        for (int k = 0; k < kV; ++k) {
            const int64_t xi = t * kTileE + threadIdx.x + (int64_t)k * kBlock;
            act[k] = xi < A.n;
            x[k] = act[k] ? (int32_t)xi : 0;
            p[k] = act[k] ? A.parent[xi] : 0;
            act[k] = act[k] && p[k] != x[k];
            q[k] = p[k];
        }
        // q[k] walks from p[k]; r[k] is the next link read
        int32_t r[kV];
#pragma unroll
        for (int k = 0; k < kV; ++k) r[k] = act[k] ? A.parent[q[k]] : q[k];
        for (int hop = 0; hop < kMaxHops; ++hop) {
            bool more = false, mv[kV];
#pragma unroll
            for (int k = 0; k < kV; ++k) {
                mv[k] = act[k] && r[k] != q[k];
                more |= mv[k];
            }
            if (!more) break;
#pragma unroll
            for (int k = 0; k < kV; ++k)
                if (mv[k]) q[k] = r[k];
#pragma unroll
            for (int k = 0; k < kV; ++k)
                if (mv[k]) r[k] = A.parent[q[k]];
        }
#pragma unroll
        for (int k = 0; k < kV; ++k) {
            if (!act[k]) continue;
            if (q[k] != p[k]) A.parent[x[k]] = q[k];
            left |= r[k] != q[k];   // stopped at the hop bound short of a root
        }
    }
    if (ballot(left) && lane_id() == 0)
        __hip_atomic_store(&A.status[kDeep], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    grid_barrier(A.bar, A.status, A.barrier_ticks);
    if (load_status(A.status) || load_status(&A.status[kDeep])) return;
    stamp(A.status, pass + 1);
    int32_t vg = -1;   // thread 0: graph of the last vertex tile's first vertex
    for (int64_t t = vw.first; t < vw.end; t += vw.step) {
        const int64_t x0 = t * kTileE;
        __syncthreads();
        if (threadIdx.x == 0) {
            if (vg < 0) vg = graph_of(A.vert_off, A.G, x0);   // then forward, as in pass 0
            else
                while (A.vert_off[vg + 1] <= x0) ++vg;
            sh_g = vg;
        }
        __syncthreads();
        int32_t g = sh_g;
        for (int64_t x = x0 + threadIdx.x; x < x0 + kTileE && x < A.n; x += kBlock) {
            while (A.vert_off[g + 1] <= x) ++g;
            A.parent[x] = (int32_t)(A.parent[x] - A.vert_off[g]);
        }
    }
}

// ------------------------------------------- fallback without a persistent grid
// Disjoint-union relabel: edge e of graph g becomes (vert_off[g] + u[e],
// vert_off[g] + v[e]); an edge with an id outside its graph becomes (-1, -1),
// which the SV pass counts as out of range.  Offsets that decrease set *bad.
__global__ __launch_bounds__(kBlock) void union_relabel_kernel(const int32_t* __restrict__ u,
                                                               const int32_t* __restrict__ v,
                                                               const int64_t* __restrict__ edge_off,
                                                               const int64_t* __restrict__ vert_off, int32_t G,
                                                               int64_t m, int32_t* __restrict__ gu,
                                                               int32_t* __restrict__ gv,
                                                               unsigned long long* __restrict__ bad) {
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t g = tid; g < G; g += stride)
        if (edge_off[g + 1] < edge_off[g] || vert_off[g + 1] < vert_off[g]) atomic_add_agent(bad, 1ull);
    for (int64_t e = tid; e < m; e += stride) {
        const int32_t g = graph_of(edge_off, G, e);
        const int64_t v0 = vert_off[g];
        const int64_t nl = vert_off[g + 1] - v0;
        const int32_t x = u[e], y = v[e];
        const bool ok = x >= 0 && y >= 0 && (int64_t)x < nl && (int64_t)y < nl;
        gu[e] = ok ? (int32_t)(v0 + x) : -1;
        gv[e] = ok ? (int32_t)(v0 + y) : -1;
    }
}

// labels[x] -= vert_off[graph of x]: global minimum ids -> graph-local labels
__global__ __launch_bounds__(kBlock) void union_unshift_kernel(int32_t* __restrict__ labels,
                                                               const int64_t* __restrict__ vert_off, int32_t G,
                                                               int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n; x += stride)
        labels[x] = (int32_t)(labels[x] - vert_off[graph_of(vert_off, G, x)]);
}

static int grid_for_items(int64_t items) {
    int64_t g = (items + 4 * kBlock - 1) / (4 * kBlock);
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (int)g;
}

hipError_t launch_union_relabel(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                                int32_t G, int64_t m, int32_t* gu, int32_t* gv, unsigned long long* bad,
                                hipStream_t s) {
    union_relabel_kernel<<<grid_for_items(m > G ? m : G), kBlock, 0, s>>>(u, v, edge_off, vert_off, G, m, gu, gv,
                                                                           bad);
    return hipGetLastError();
}

hipError_t launch_union_unshift(int32_t* labels, const int64_t* vert_off, int32_t G, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    union_unshift_kernel<<<grid_for_items(n), kBlock, 0, s>>>(labels, vert_off, G, n);
    return hipGetLastError();
}

hipError_t batched_max_blocks(int* blocks) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel, kBlock, 0);
    if (e != hipSuccess) return e;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // The grid barrier needs every workgroup resident at once.  A grid at the
    // full occupancy bound was accepted by the cooperative launch but did not
    // all become resident on gfx950 (the barrier's timeout fired), so stay at
    // half of it and at most 4 workgroups per CU.
    int b = per_cu * cus / 2;
    if (b > 4 * cus) b = 4 * cus;
    *blocks = b > 0 ? b : 1;
    return hipSuccess;
}

hipError_t launch_batched(const BatchArgsHost& h, int blocks, hipStream_t s) {
    BatchArgs A;
    A.u = h.u;
    A.v = h.v;
    A.edge_off = h.edge_off;
    A.vert_off = h.vert_off;
    A.G = h.G;
    A.m = h.m;
    A.n = h.n;
    A.parent = h.labels;
    A.buf0 = h.buf0;
    A.buf1 = h.buf1;
    A.cnt0 = h.cnt0;
    A.cnt1 = h.cnt1;
    A.hcnt = h.hcnt;
    A.hooked = h.hooked;
    A.bar = h.bar;
    A.status = h.status;
    A.max_passes = h.max_passes;
    A.max_link = h.max_link;
    A.barrier_ticks = h.barrier_ticks;
    A.part = h.part;
    A.bstat = h.bstat;
    void* args[] = {&A};
    return hipLaunchCooperativeKernel((const void*)batched_kernel, dim3(blocks), dim3(kBlock), args, 0, s);
}

}  // namespace ccmi
