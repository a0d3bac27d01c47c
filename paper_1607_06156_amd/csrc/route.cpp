// Route selection and the hybrid driver of Algorithm 2 (Section III-B).
//
//   prediction : degree distribution (bucketed degree pass + histograms);
//   decision   : K-S statistic of the power-law fit < tau -> BFS step, or the
//                learned router's argmax;
//   BFS step   : CSR, direction-optimising BFS from the max-degree vertex,
//                component label, edge filter;
//   SV         : the SV iteration on whatever edges remain.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "bfs.hpp"
#include "degree.hpp"
#include "internal.hpp"
#include "ks.hpp"
#include "router.hpp"

namespace ccmi {

static int sync_read(Call& c, void* host, const void* dev, size_t bytes) {
    hipError_t e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(D2H)");
    e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return CC_OK;
}

// ------------------------------------------------------------ prediction
// WS_CURSOR holds, one after the other in time, the first level of the
// two-level scatter (uint32 ids, + int32 other ends for a CSR) and the CSR
// fill's regrouped entries (uint16 ids, int32 other ends).
static size_t cursor_bytes(int64_t m, bool csr) {
    return csr ? (size_t)2 * m * 8 : (size_t)2 * m * 4;
}

static void set_cursor_bufs(BucketBufs* w, void* po, int64_t m, bool csr) {
    w->loc32 = (uint32_t*)po;
    w->other32 = po && csr ? (int32_t*)((uint32_t*)po + 2 * m) : nullptr;
    w->tloc = csr ? (uint16_t*)po : nullptr;
    w->tother = po && csr ? (int32_t*)((char*)po + (((size_t)2 * m * sizeof(uint16_t) + 255) & ~(size_t)255))
                          : nullptr;
}

// Pinned staging of the degree pass's readback: the histograms and counters
// at the start, the tail prefetch (up to kTailPrefetch entries) at this offset.
constexpr size_t kTailPrefetchOff = 64 * 1024;
constexpr int64_t kTailPrefetch = 16 * 1024;
static_assert((64 + kExactBins + 4) * sizeof(unsigned long long) <= kTailPrefetchOff, "staging overlap");
static_assert(kTailPrefetchOff + kTailPrefetch * sizeof(int32_t) <= Workspace::kHostBytes, "staging size");

int run_degree_pass(Call& c, bool want_csr, DegreeResult* r) {
    Workspace& ws = *c.ws;
    BucketPlan p;
    if (c.m >= (int64_t)1 << 31) return fail(CC_EINVAL, "m too large for the degree pass (m < 2^31)");
    if (bucket_plan(c.n, c.m, &p)) return fail(CC_EINVAL, "n too large for the degree pass");
    r->plan = p;
    const int64_t m = c.m;
    void *pc, *po, *pp, *pdeg, *ptail;
    int rc;
    // WS_HIST: per-block bucket counts, then (8-byte aligned) totals, bases,
    // error counter, then the CSR fill's per-group counters
    const size_t counts_bytes = ((size_t)p.nblk * p.B * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t tot_bytes = (size_t)(2 * p.B + 3) * sizeof(unsigned long long);
    if ((rc = ws.get(WS_HIST, counts_bytes + tot_bytes + (size_t)p.B * kGroups * sizeof(uint32_t), &pc))) return rc;
    if (p.B > kStagedMaxB || want_csr) {
        // the first level of the two-level scatter (32-bit ids, + other ends
        // for a CSR) and, later, the CSR fill's regrouped entries share it
        if ((rc = ws.get(WS_CURSOR, cursor_bytes(m, want_csr), &po))) return rc;
    } else {
        po = nullptr;
    }
    // bucketed endpoints: 16-bit local ids, then (256-aligned) the other ends
    const size_t loc_bytes = ((size_t)2 * m * sizeof(uint16_t) + 255) & ~(size_t)255;
    if ((rc = ws.get(WS_QUEUE, loc_bytes + (size_t)2 * m * sizeof(int32_t), &pp))) return rc;
    if ((rc = ws.get(WS_DEG, (size_t)c.n * sizeof(int32_t), &pdeg))) return rc;
    const int64_t tail_cap = std::min<int64_t>(c.n, 2 * m / kExactBins + 1);
    if ((rc = ws.get(WS_TAIL, (size_t)tail_cap * sizeof(int32_t), &ptail))) return rc;
    BucketBufs w;
    w.counts = (uint32_t*)pc;
    w.tot = (unsigned long long*)((char*)pc + counts_bytes);
    w.base = w.tot + p.B;
    w.err = w.base + p.B + 1;
    w.gcnt = (uint32_t*)((char*)pc + counts_bytes + tot_bytes);
    set_cursor_bufs(&w, po, m, want_csr);
    w.loc = (uint16_t*)pp;
    w.other = (int32_t*)((char*)pp + loc_bytes);
    // without a CSR the other ends' space is free: the capped layout may use it
    w.loc_cap = want_csr ? 2 * m : (int64_t)((loc_bytes + (size_t)2 * m * sizeof(int32_t)) / sizeof(uint16_t));
    r->bufs = w;
    r->deg = c.deg_out ? c.deg_out : (int32_t*)pdeg;
    r->tail = (int32_t*)ptail;
    r->tail_cap = tail_cap;
    // WS_HISTOUT: hist64[64], histx[4096], tail count, arg-max key
    void* ph;
    if ((rc = ws.get(WS_HISTOUT, (64 + kExactBins + 4) * sizeof(unsigned long long), &ph))) return rc;
    unsigned long long* hist64 = (unsigned long long*)ph;
    unsigned long long* histx = hist64 + 64;
    unsigned long long* tail_count = histx + kExactBins;
    unsigned long long* argmax_key = tail_count + 1;
    r->hist64_dev = hist64;
    hipError_t e;
    int64_t* off = nullptr;
    int32_t* adj = nullptr;
    if (want_csr) {
        if (c.off_out && c.adj_out) {
            off = c.off_out;
            adj = c.adj_out;
        } else {
            void *poff, *padj;
            if ((rc = ws.get(WS_OFF, (size_t)(c.n + 1) * sizeof(int64_t), &poff))) return rc;
            if ((rc = ws.get(WS_ADJ, (size_t)2 * m * sizeof(int32_t), &padj))) return rc;
            off = (int64_t*)poff;
            adj = (int32_t*)padj;
        }
        r->off = off;
        r->adj = adj;
    }
    unsigned long long* host;
    if ((rc = ws.pinned((void**)&host))) return rc;
    // The capped layout (no count pass) first; if one of its runs overflowed
    // (a hub far above its bucket's share), the counted layout again.
    for (int attempt = 0;; ++attempt) {
    e = hipMemsetAsync(ph, 0, (64 + kExactBins + 4) * sizeof(unsigned long long), c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(w.err, 0, 2 * sizeof(unsigned long long), c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    int k0 = c.kbeg();
    e = launch_bucket_degree(c.u, c.v, m, c.n, p, w, r->deg, 1, hist64, histx, r->tail, tail_cap, tail_count,
                             argmax_key, want_csr ? 1 : 0, off, adj, c.stream, attempt == 0);
    if (e != hipSuccess) return hip_fail(e, "degree pass launch");
    r->bufs = w;
    // algorithmic bytes: edges read (8 B), degrees written and histogrammed (8 B per vertex),
    // plus the CSR (8 B per adjacency entry written, 8 B per offset)
    c.kend(CC_K_DEGREE, k0, 8.0 * m + 8.0 * c.n + (want_csr ? 16.0 * m + 8.0 * c.n : 0.0));
    if (c.stats) c.bytes += 8.0 * m + 8.0 * c.n + (want_csr ? 16.0 * m + 8.0 * c.n : 0.0);
    r->csr_built = want_csr;
    // read back histograms + counters
    e = hipMemcpyAsync(host, ph, (64 + kExactBins + 2) * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                       c.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host + 64 + kExactBins + 2, w.err, 2 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, c.stream);
    // the route decision needs the tail too: its first entries come back in
    // the same round trip (the tail count is not known before it)
    r->tail_host = nullptr;
    r->tail_host_n = 0;
    if (e == hipSuccess && r->prefetch_tail) {
        r->tail_host_n = std::min<int64_t>(tail_cap, kTailPrefetch);
        r->tail_host = (const int32_t*)((char*)host + kTailPrefetchOff);
        e = hipMemcpyAsync((void*)r->tail_host, r->tail, (size_t)r->tail_host_n * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c.stream);
    }
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(hist)");
    if (r->spec && !r->spec->launched) {
        // The SV route's first launch goes in behind the readback, so the GPU
        // labels while the host fits the degree distribution; only the
        // readback is waited for.
        hipEvent_t ev;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        e = hipEventRecord(ev, c.stream);
        SvInput in;
        in.soa = true;
        in.u = c.u;
        in.v = c.v;
        in.m = c.m;
        rc = e == hipSuccess ? sv_speculate(c, in, r->spec) : CC_OK;
        if (e == hipSuccess) e = hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        if (rc) return rc;
    } else {
        e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    if (host[64 + kExactBins + 3] == 0 || attempt > 0) break;
    }
    if (host[64 + kExactBins + 2])
        return fail(CC_ERANGE, "%llu edges have an endpoint outside [0, n)", host[64 + kExactBins + 2]);
    for (int i = 0; i < 64; ++i) r->hist64[i] = (int64_t)host[i];
    r->histx.assign(host + 64, host + 64 + kExactBins);
    r->ntail = (int64_t)host[64 + kExactBins];
    const unsigned long long key = host[64 + kExactBins + 1];
    r->max_degree = (int64_t)(key >> 32);
    r->argmax = r->max_degree > 0 ? (int32_t)(~(uint32_t)(key & 0xffffffffull)) : -1;
    c.range_checked = true;
    if (c.stats) c.stats->max_degree = r->max_degree;
    return CC_OK;
}

int decide_heuristic(Call& c, DegreeResult& r, int* route) {
    // the tail list comes back through the pinned staging buffer when it fits
    // (ks_fit copies it before it reuses that buffer)
    std::vector<int32_t> pageable;
    const int32_t* tail = nullptr;
    int64_t ntail = 0;
    if (r.ntail > 0 && std::min(r.ntail, r.tail_cap) <= r.tail_host_n) {
        // read back with the histograms already
        ntail = std::min(r.ntail, r.tail_cap);
        tail = r.tail_host;
    } else if (r.ntail > 0) {
        ntail = std::min(r.ntail, r.tail_cap);
        int32_t* dst;
        if ((size_t)ntail * sizeof(int32_t) <= Workspace::kHostBytes) {
            void* hp;
            int rc = c.ws->pinned(&hp);
            if (rc) return rc;
            dst = (int32_t*)hp;
        } else {
            pageable.resize(ntail);
            dst = pageable.data();
        }
        hipError_t e = hipMemcpyAsync(dst, r.tail, ntail * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tail)");
        e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        tail = dst;
    }
    // With a speculative SV launch in the call's stream, the fit goes to the
    // second stream and runs beside it.  Its inputs come from the host and its
    // scratch is WS_KS, which that launch does not touch; a stream-ordered
    // pool allocation belongs to the call's stream, so that mode keeps it.
    hipStream_t ks_s = c.stream;
    if (r.spec && r.spec->launched && c.ws->mode != Workspace::kPool) {
        hipStream_t side;
        if (side_stream(&side) == CC_OK) ks_s = side;
    }
    KsResult k;
    int rc = ks_fit(*c.ws, ks_s, r.histx.data(), tail, ntail, &k);
    if (rc) return rc;
    if (c.stats) {
        c.stats->ks_statistic = k.ks;
        c.stats->ks_alpha = k.alpha;
        c.stats->ks_dmin = k.dmin;
    }
    r.hub_min = k.hub_min;
    *route = (k.ks < c.opt.tau) ? CC_R0_BFS_SV : CC_R1_SV;
    return CC_OK;
}

// ------------------------------------------------------------------- BFS
int run_bfs(Call& c, const int64_t* off, const int32_t* adj, int64_t nadj, int32_t seed, int64_t seed_deg,
            int max_levels, uint32_t** vis_out, BfsResult* br) {
    Workspace& ws = *c.ws;
    const int32_t n = c.n;
    const int64_t words = ((int64_t)n + 31) >> 5;
    void *pbits, *pq, *ppre, *ptot;
    int rc;
    if ((rc = ws.get(WS_BITS, (size_t)words * 3 * sizeof(uint32_t), &pbits))) return rc;
    if ((rc = ws.get(WS_HOOKED, (size_t)n * 2 * sizeof(int32_t), &pq))) return rc;
    const int64_t nb = ((int64_t)n + 1023) / 1024 + 1;
    if ((rc = ws.get(WS_SEGCOUNT, (size_t)(n + 1 + nb + 1) * sizeof(int64_t), &ppre))) return rc;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &ptot))) return rc;
    uint32_t* vis = (uint32_t*)pbits;
    uint32_t* front = vis + words;
    uint32_t* next = front + words;
    int32_t* q = (int32_t*)pq;
    int32_t* nq = q + n;
    int64_t* pre = (int64_t*)ppre;
    int64_t* bsum = pre + n + 1;
    int64_t* qtot = bsum + nb;
    unsigned long long* ctr = (unsigned long long*)ptot + 16;
    unsigned long long* host;
    if ((rc = ws.pinned((void**)&host))) return rc;
    hipError_t e = hipMemsetAsync(vis, 0, words * sizeof(uint32_t), c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(vis)");
    int32_t* hs = (int32_t*)(host + 32);
    hs[0] = seed;
    e = hipMemcpyAsync(q, hs, sizeof(int32_t), hipMemcpyHostToDevice, c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(seed)");
    if ((e = launch_queue_to_bits(q, 1, vis, c.stream)) != hipSuccess) return hip_fail(e, "seed bit");
    int64_t qn = 1, nf = 1, mf = seed_deg, mu = 2 * c.m - seed_deg, prev_nf = 0;
    int64_t visited = 1, examined = 0;
    bool topdown = true;
    int levels = 0, bu_levels = 0;
    while (nf > 0) {
        if (topdown && mf <= kFewLevelEntries) {
            // small frontiers: as many levels as stay small in one workgroup,
            // one launch and one readback for all of them
            const int budget = max_levels > 0 ? max_levels - levels : INT32_MAX;
            int k0 = c.kbeg();
            if ((e = launch_bfs_few(off, adj, q, nq, qn, kFewLevelEntries, budget, vis, pre, ctr, c.stream)) !=
                hipSuccess)
                return hip_fail(e, "bfs_few launch");
            int rec = c.kend(CC_K_BFS, k0, 0.0);
            if ((rc = sync_read(c, host, ctr, 6 * sizeof(unsigned long long)))) return rc;
            const int lr = (int)host[0];
            if (lr < 1) {
                // the frontier's entries exceed what the host counted: expand
                // it with the launch-per-level code below
                mf = (int64_t)host[5];
                if (mf <= kFewLevelEntries) return fail(CC_EINTERNAL, "BFS made no progress on a small frontier");
                goto multi;
            }
            // per level: queue and offsets of the frontier (scan and walk),
            // entries, bitmap probes, new vertices' offsets and queue slots
            const double lbytes = 28.0 * (double)host[1] + 8.0 * (double)host[2];
            c.kbytes(rec, lbytes);
            if (c.stats) c.bytes += lbytes;
            levels += lr;
            visited += (int64_t)host[1];
            examined += (int64_t)host[2];
            mu -= (int64_t)host[3];
            prev_nf = nf;
            nf = qn = (int64_t)host[4];
            mf = (int64_t)host[5];
            if (max_levels > 0 && levels >= max_levels && nf > 0) {
                br->abandoned = true;
                break;
            }
            continue;
        }
    multi:
        if (topdown && (double)mf > (double)mu / kBeamerAlpha) {
            // switch to bottom-up: frontier queue -> bitmap
            if ((e = hipMemsetAsync(front, 0, words * sizeof(uint32_t), c.stream)) != hipSuccess)
                return hip_fail(e, "hipMemsetAsync(front)");
            if ((e = launch_queue_to_bits(q, qn, front, c.stream)) != hipSuccess) return hip_fail(e, "q2b");
            topdown = false;
        }
        if ((e = hipMemsetAsync(ctr, 0, 4 * sizeof(unsigned long long), c.stream)) != hipSuccess)
            return hip_fail(e, "hipMemsetAsync(ctr)");
        int k0 = c.kbeg();
        if (topdown) {
            if ((e = launch_qdeg_scan(q, qn, off, pre, bsum, qtot, c.stream)) != hipSuccess)
                return hip_fail(e, "qdeg scan");
            if ((e = launch_topdown(q, qn, pre, mf, off, adj, vis, nq, ctr, c.stream)) != hipSuccess)
                return hip_fail(e, "topdown");
        } else {
            if ((e = launch_bottomup(n, off, adj, vis, front, next, ctr, c.stream)) != hipSuccess)
                return hip_fail(e, "bottomup");
        }
        int rec = c.kend(CC_K_BFS, k0, 0.0);
        if ((rc = sync_read(c, host, ctr, 3 * sizeof(unsigned long long)))) return rc;
        const int64_t found = (int64_t)host[0], fdeg = (int64_t)host[1];
        double lbytes;
        if (topdown) {
            // queue + offsets of the frontier, adjacency entries, bitmap probes, queue writes
            lbytes = 20.0 * qn + 8.0 * mf + 8.0 * found;
            examined += mf;
            std::swap(q, nq);
            qn = found;
        } else {
            // offsets of unvisited vertices, entries examined, bitmap words in/out
            const int64_t exam = (int64_t)host[2];
            lbytes = 16.0 * (n - visited) + 8.0 * exam + 12.0 * words;
            examined += exam;
            std::swap(front, next);
            ++bu_levels;
        }
        c.kbytes(rec, lbytes);
        if (c.stats) c.bytes += lbytes;
        ++levels;
        visited += found;
        mu -= fdeg;
        prev_nf = nf;
        nf = found;
        mf = fdeg;
        if (!topdown && nf > 0 && (double)nf < (double)n / kBeamerBeta && nf < prev_nf) {
            // frontier shrinking: back to top-down, bitmap -> queue
            if ((e = hipMemsetAsync(ctr + 3, 0, sizeof(unsigned long long), c.stream)) != hipSuccess)
                return hip_fail(e, "hipMemsetAsync");
            if ((e = launch_bits_to_queue(front, words, q, ctr + 3, c.stream)) != hipSuccess) return hip_fail(e, "b2q");
            if ((rc = sync_read(c, host, ctr + 3, sizeof(unsigned long long)))) return rc;
            qn = (int64_t)host[0];
            topdown = true;
        }
        if (max_levels > 0 && levels >= max_levels && nf > 0) {
            br->abandoned = true;
            break;
        }
    }
    (void)nadj;
    br->unvisited_entries = mu;   // 2m minus the degrees of the visited vertices
    br->levels = levels;
    br->bottom_up = bu_levels;
    br->visited = visited;
    br->examined = examined;
    *vis_out = vis;
    return CC_OK;
}

// The BFS step is meant for a short-diameter component (Section III-B): each
// level costs a launch and a host round trip, so a long path would cost one per
// hop.  A BFS still running after this many levels is abandoned before any
// label is written, and SV labels the whole graph instead.
constexpr int kMaxBfsLevels = 256;

// R0: CSR (if not built yet), BFS, label, filter, then SV on the rest
int run_bfs_route(Call& c, DegreeResult& r) {
    Workspace& ws = *c.ws;
    int rc;
    int t0 = c.timer->mark();
    if (!r.csr_built) {
        void *poff, *padj;
        if ((rc = ws.get(WS_OFF, (size_t)(c.n + 1) * sizeof(int64_t), &poff))) return rc;
        if ((rc = ws.get(WS_ADJ, (size_t)2 * c.m * sizeof(int32_t), &padj))) return rc;
        r.off = (int64_t*)poff;
        r.adj = (int32_t*)padj;
        if (!r.bufs.other_written) {
            // the scatter runs again with the other ends, then the fill
            void* po;
            if ((rc = ws.get(WS_CURSOR, cursor_bytes(c.m, true), &po))) return rc;
            set_cursor_bufs(&r.bufs, po, c.m, true);
        }
        int k0 = c.kbeg();
        hipError_t e = launch_bucket_csr_from_deg(c.u, c.v, c.m, c.n, r.plan, r.bufs, r.deg, r.off, r.adj, c.stream);
        if (e != hipSuccess) return hip_fail(e, "csr launch");
        c.kend(CC_K_CSR, k0, 16.0 * c.m + 12.0 * c.n);
        if (c.stats) c.bytes += 16.0 * c.m + 12.0 * c.n;
        r.csr_built = true;
    }
    int t1 = c.timer->mark();
    uint32_t* vis = nullptr;
    BfsResult br{};
    rc = run_bfs(c, r.off, r.adj, 2 * c.m, r.argmax, r.max_degree, kMaxBfsLevels, &vis, &br);
    if (rc) return rc;
    int t2 = c.timer->mark();
    if (br.abandoned) {
        if (c.stats) {
            c.stats->route = CC_R1_SV;
            c.stats->bfs_levels = br.levels;
            c.stats->bfs_bottom_up_levels = br.bottom_up;
            c.stats->bfs_seed = r.argmax;
            c.stats->bfs_visited = br.visited;
            c.stats->bfs_edges_examined = br.examined;
            c.stats->ms_csr = c.timer->ms(t0, t1);
            c.stats->ms_bfs = c.timer->ms(t1, t2);
        }
        SvInput in;
        in.soa = true;
        in.u = c.u;
        in.v = c.v;
        in.m = c.m;
        int t4 = c.timer->mark();
        rc = run_sv(c, in, CC_R1_SV, c.opt.theta, c.opt.max_passes);
        if (c.stats) c.stats->ms_sv = c.timer->ms(t4, c.timer->mark());
        return rc;
    }
    // label + filter
    void *ptot, *pe0, *pcnt;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &ptot))) return rc;
    unsigned long long* tot = (unsigned long long*)ptot + 24;
    int32_t* dlabel = (int32_t*)((unsigned long long*)ptot + 28);
    const int nseg = choose_nseg(c.m);
    const int64_t cap = (c.m + nseg - 1) / nseg;
    // the size run_sv asks for (7 words per segment), so that the filtered
    // list's counts stay where they are when SV takes the list over
    if ((rc = ws.get(WS_SEGCOUNT, std::max((size_t)nseg * 7 * sizeof(uint32_t),
                                           (size_t)(c.n + 1 + c.n / 1024 + 3) * sizeof(int64_t)),
                     &pcnt)))
        return rc;
    // The rest is read from the CSR rows of the unvisited vertices when they
    // hold no more entries than the edge list has edges (typically a few
    // percent after a giant component): half the bytes at most, and no bitmap
    // probe per edge.  Otherwise every edge of the list is tested.
    const bool from_csr = br.unvisited_entries <= c.m;
    int k0 = c.kbeg();
    hipError_t e = hipMemsetAsync(dlabel, 0x7f, sizeof(int32_t), c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(tot + 1, 0, sizeof(unsigned long long), c.stream);
    if (e == hipSuccess) e = launch_bfs_label(vis, c.n, dlabel, c.parent, c.stream);
    SegList out{};
    int64_t* wcount = (int64_t*)pcnt;
    if (from_csr) {
        if (e == hipSuccess) e = launch_rest_count(vis, r.off, r.adj, c.n, wcount, (int64_t*)tot, c.stream);
    } else {
        if ((rc = ws.get(WS_EDGES0, (size_t)nseg * cap * sizeof(int2), &pe0))) return rc;
        uint32_t* fcnt = (uint32_t*)pcnt + (size_t)2 * nseg;
        out = SegList{(int2*)pe0, cap, nseg, fcnt};
        if (e == hipSuccess) e = launch_filter(c.u, c.v, c.m, c.n, vis, out, tot, tot + 1, c.stream);
    }
    if (e != hipSuccess) return hip_fail(e, "label/filter launch");
    int rec = c.kend(CC_K_FILTER, k0, 0.0);
    unsigned long long* host;
    if ((rc = ws.pinned((void**)&host))) return rc;
    e = hipMemcpyAsync(host, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host + 1, dlabel, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "filter readback");
    const int64_t kept = (int64_t)host[0];
    const int32_t label = *(int32_t*)(host + 1);
    int32_t* fu = nullptr;
    int32_t* fv = nullptr;
    double fbytes;
    if (from_csr) {
        // the rest as dense arrays in the CSR fill's scratch (free by now)
        void* pf;
        if ((rc = ws.get(WS_CURSOR, (size_t)std::max<int64_t>(kept, 1) * 2 * sizeof(int32_t), &pf))) return rc;
        fu = (int32_t*)pf;
        fv = fu + kept;
        if (kept > 0) {
            int k1 = c.kbeg();
            e = launch_rest_emit(vis, r.off, r.adj, c.n, wcount, fu, fv, c.stream);
            if (e != hipSuccess) return hip_fail(e, "rest launch");
            c.kend(CC_K_FILTER, k1, 0.125 * c.n + 16.0 * (c.n - br.visited) + 4.0 * br.unvisited_entries +
                                        8.0 * kept);
        }
        // labels (4 B per vertex), bitmap, offsets of the unvisited vertices, their rows (counted)
        fbytes = 4.0 * c.n + 0.25 * c.n + 16.0 * (c.n - br.visited) + 4.0 * br.unvisited_entries;
    } else {
        // labels (4 B per vertex) + bitmap probe per vertex and per edge, edges read, survivors written
        fbytes = 4.0 * c.n + 0.125 * c.n + 8.0 * c.m + 4.0 * c.m + 8.0 * kept;
    }
    c.kbytes(rec, fbytes);
    if (c.stats) {
        c.bytes += fbytes + (from_csr && kept > 0 ? 0.125 * c.n + 16.0 * (c.n - br.visited) +
                                                         4.0 * br.unvisited_entries + 8.0 * kept
                                                   : 0.0);
        c.stats->bfs_levels = br.levels;
        c.stats->bfs_bottom_up_levels = br.bottom_up;
        c.stats->bfs_seed = r.argmax;
        c.stats->bfs_label = label;
        c.stats->bfs_visited = br.visited;
        c.stats->bfs_edges_examined = br.examined;
        c.stats->edges_after_filter = kept;
    }
    int t3 = c.timer->mark();
    if (c.stats) {
        c.stats->ms_csr = c.timer->ms(t0, t1);
        c.stats->ms_bfs = c.timer->ms(t1, t2);
        c.stats->ms_filter = c.timer->ms(t2, t3);
    }
    if (kept == 0) return CC_OK;
    SvInput in;
    if (from_csr) {
        in.soa = true;
        in.u = fu;
        in.v = fv;
        in.m = kept;
    } else {
        in.soa = false;
        in.m = kept;
        in.seg = out;
    }
    int t4 = c.timer->mark();
    rc = run_sv(c, in, CC_R1_SV, c.opt.theta, c.opt.max_passes);
    int t5 = c.timer->mark();
    if (c.stats) c.stats->ms_sv = c.timer->ms(t4, t5);
    return rc;
}

// --------------------------------------------------------------- driver
int run_label(Call& c) {
    int k0 = c.kbeg();
    hipError_t e = launch_sv_init(c.parent, c.n, c.stream);
    if (e != hipSuccess) return hip_fail(e, "sv_init launch");
    c.kend(CC_K_SV_FINALIZE, k0, 4.0 * c.n);
    if (c.stats) c.bytes += 4.0 * c.n;
    if (c.m == 0) {
        if (c.stats) c.stats->route = CC_R1_SV;
        return CC_OK;
    }
    int req = c.opt.route;
    if (req == CC_ROUTE_AUTO) req = router_loaded() ? CC_ROUTE_ROUTER : CC_ROUTE_HEURISTIC;
    if (req == CC_ROUTE_ROUTER && !router_loaded()) return fail(CC_ENOROUTER, "no router weights loaded");
    BucketPlan probe;
    const bool can_predict = bucket_plan(c.n, c.m, &probe) == 0 && c.m < (int64_t)1 << 31;
    int route = CC_R1_SV;
    DegreeResult dr;
    SvSpec spec;
    int rc;
    int tp0 = c.timer->mark();
    if (req == CC_ROUTE_SV) route = CC_R1_SV;
    else if (req == CC_ROUTE_SV_THETA) route = CC_R2_SV_THETA;
    else if (!can_predict) route = CC_R1_SV;   // beyond the bucketed pass: SV handles any size
    else if (req == CC_ROUTE_BFS_SV) {
        if ((rc = run_degree_pass(c, true, &dr))) return rc;
        route = CC_R0_BFS_SV;
    } else {
        // the SV route's first launch runs while the host decides (sv_speculate)
        dr.prefetch_tail = req == CC_ROUTE_HEURISTIC;
        dr.spec = &spec;
        rc = run_degree_pass(c, false, &dr);
        if (rc == CC_OK) rc = req == CC_ROUTE_HEURISTIC ? decide_heuristic(c, dr, &route) : decide_router(c, dr, &route);
        if (rc) {
            if (spec.launched) (void)hipStreamSynchronize(c.stream);   // no kernel outlives the call
            return rc;
        }
    }
    int tp1 = c.timer->mark();
    // the speculative launch counts as SV time, not prediction
    const double spec_ms = spec.launched ? c.timer->ms(spec.t0, spec.t1) : 0.0;
    if (c.stats) {
        c.stats->route = route;
        c.stats->ms_predict = c.timer->ms(tp0, tp1) - spec_ms;
    }
    if (route == CC_R0_BFS_SV) {
        if (dr.argmax < 0) {
            route = CC_R1_SV;   // no edge with a valid endpoint: nothing to traverse
        } else {
            if (spec.launched) {
                // the BFS route starts from single vertices: undo the speculative hooks
                hipError_t e = launch_sv_init(c.parent, c.n, c.stream);
                if (e != hipSuccess) return hip_fail(e, "sv_init launch");
            }
            return run_bfs_route(c, dr);
        }
    }
    if (dr.deg && dr.hub_min > 0 && dr.hub_min < INT32_MAX) {
        c.hub_deg = dr.deg;
        c.hub_min = (int32_t)dr.hub_min;
    }
    SvInput in;
    in.soa = true;
    in.u = c.u;
    in.v = c.v;
    in.m = c.m;
    int t0 = c.timer->mark();
    rc = run_sv(c, in, route, c.opt.theta, c.opt.max_passes, &spec);
    int t1 = c.timer->mark();
    if (c.stats) c.stats->ms_sv = c.timer->ms(t0, t1) + spec_ms;
    return rc;
}

}  // namespace ccmi
