// Host side of batched labelling: validation, workspace, the autotuner and
// the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batched.hpp"
#include "common.hpp"
#include "internal.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

constexpr size_t kBatchCtl = 1024;      // barrier words + status block
constexpr int kStatusWords = 48;        // status[0..3) codes, [4] deep chains left, status[8..48) pass stamps
constexpr int kStatusDeep = 4;
// host staging: the status words at 0, the per-block counts (4 x blocks,
// blocks <= 16384) from this word on
constexpr size_t kBstatHost = 1024;
static_assert((kBstatHost + 4 * 16384) * sizeof(unsigned long long) <= Workspace::kHostBytes, "staging size");
// status[0] error bits written by the persistent kernel
constexpr unsigned long long kErrRangeBit = 1, kErrOffsetsBit = 2, kErrBarrierBit = 4;
// default spin limit of the kernel's grid barrier: 5 s of the 100 MHz wall clock
constexpr uint64_t kBarrierTicks = 500000000ull;

// CC_BATCH_BARRIER_TICKS (a positive integer) overrides the spin limit, so the
// fallback that a barrier timeout takes can be exercised from the host.
static uint64_t barrier_ticks() {
    const char* s = getenv("CC_BATCH_BARRIER_TICKS");
    if (!s || !*s) return kBarrierTicks;
    char* end = nullptr;
    unsigned long long t = strtoull(s, &end, 10);
    return (end && *end == 0 && t > 0) ? (uint64_t)t : kBarrierTicks;
}

// The persistent kernel's final compression met a chain deeper than one walk
// (kMaxHops links) and left the labels as global, unflattened parents: flatten
// rounds until every vertex points at its root, then shift to graph-local
// labels.  ctl: the kernel's control block (the round flag sits at +512);
// hw: pinned host words (hw[kStatusWords] is used).
static int finish_deep(const BatchArgsHost& h, void* ctl, unsigned long long* hw, hipStream_t s) {
    unsigned long long* open = (unsigned long long*)((char*)ctl + 512);
    for (int r = 0;; ++r) {
        if (r >= 16) return fail(CC_EINTERNAL, "flatten did not finish");
        hipError_t e = hipMemsetAsync(open, 0, sizeof(*open), s);
        if (e == hipSuccess) e = launch_sv_finalize(h.labels, h.n, open, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hw + kStatusWords, open, sizeof(*open), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "batched flatten");
        if (!hw[kStatusWords]) break;
    }
    hipError_t e = launch_union_unshift(h.labels, h.vert_off, h.G, h.n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? CC_OK : hip_fail(e, "union unshift");
}

// ------------------------------------------------------------ autotuner
// Chooses the persistent grid size (edges per workgroup segment) and the hook
// attempts per edge and pass, per size class, by timing the candidates on the
// first call of that class.  Every candidate computes the same labels.
// Results live in memory and, if CC_AUTOTUNE_CACHE names a file, on disk (one
// "key blocks link" triple per line).
struct Tuned {
    int blocks = 0;
    int link = 1;
};
static std::mutex g_tune_mu;
static std::map<std::string, Tuned> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(int dev, int64_t m, int32_t n, int32_t G) {
    hipDeviceProp_t p;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) arch = p.gcnArchName;
    for (auto& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    char buf[256];
    snprintf(buf, sizeof buf, "%s/batched/m2^%d/n2^%d/G2^%d", arch.c_str(), (int)std::log2((double)m + 1),
             (int)std::log2((double)n + 1), (int)std::log2((double)G + 1));
    return buf;
}

static void tune_load() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = getenv("CC_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char key[256];
    int b, l;
    while (fscanf(f, "%255s %d %d", key, &b, &l) == 3) g_tune[key] = Tuned{b, l};
    fclose(f);
}

static void tune_store(const std::string& key, Tuned t) {
    g_tune[key] = t;
    const char* path = getenv("CC_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "w");
    if (!f) return;
    for (auto& kv : g_tune) fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.blocks, kv.second.link);
    fclose(f);
}

// A cooperative launch can be refused although the grid fits: the device's
// global wave-sync resource is held by another process that made cooperative
// launches on the same GPU, or the runtime cannot make the grid resident.
static bool coop_refused(hipError_t e) {
    return e == hipErrorIllegalState || e == hipErrorCooperativeLaunchTooLarge || e == hipErrorNotSupported;
}

// *refused (if given) reports a refused cooperative launch instead of an error.
static int run_once(Workspace& ws, BatchArgsHost h, int blocks, int link, hipStream_t s,
                    unsigned long long* status_host, double* ms, bool* refused) {
    const int64_t tiles = h.m > 0 ? (h.m + kBatchTile - 1) / kBatchTile : 1;
    const size_t slots = (size_t)tiles * (size_t)kBatchTile;
    void *p0, *p1, *ph, *pc, *pb;
    int rc;
    if ((rc = ws.get(WS_EDGES0, slots * sizeof(int2), &p0))) return rc;
    if ((rc = ws.get(WS_EDGES1, slots * sizeof(int2), &p1))) return rc;
    if ((rc = ws.get(WS_HOOKED, slots * sizeof(int32_t), &ph))) return rc;
    const size_t cnt_bytes = ((size_t)tiles * 3 * sizeof(uint32_t) + 255) & ~(size_t)255;
    // per-tile counts, then per-block partials (survivors, hooks and finds
    // stopped at the hop bound, two arrays each)
    if ((rc = ws.get(WS_SEGCOUNT, cnt_bytes + (size_t)blocks * 10 * sizeof(unsigned long long), &pc))) return rc;
    if ((rc = ws.get(WS_BATCH, kBatchCtl, &pb))) return rc;
    h.buf0 = (int2*)p0;
    h.buf1 = (int2*)p1;
    h.hooked = (int32_t*)ph;
    h.cnt0 = (uint32_t*)pc;
    h.cnt1 = h.cnt0 + tiles;
    h.hcnt = h.cnt1 + tiles;
    h.part = (unsigned long long*)((char*)pc + cnt_bytes);
    h.bstat = h.part + (size_t)blocks * 6;
    h.bar = (unsigned int*)pb;
    h.status = (unsigned long long*)((char*)pb + 64);
    h.max_link = link;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
    }
    hipError_t e = hipMemsetAsync(pb, 0, kBatchCtl, s);
    if (e == hipSuccess && ms) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        e = launch_batched(h, blocks, s);
        if (e != hipSuccess && refused && coop_refused(e)) {
            (void)hipGetLastError();   // clear the launch error
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            *refused = true;
            return CC_OK;
        }
    }
    if (e == hipSuccess && ms) e = hipEventRecord(e1, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(status_host, h.status, kStatusWords * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s);
    // the per-block counts of the byte model, behind the status words
    if (e == hipSuccess)
        e = hipMemcpyAsync(status_host + kBstatHost, h.bstat, (size_t)blocks * 4 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && ms) {
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    // A grid barrier that waited past its limit means that not every
    // workgroup of the grid was resident at once (the cooperative launch
    // does not stop kernels of other streams or processes from holding CUs).
    // Every workgroup has exited, and the disjoint-union fallback
    // re-initialises the labels, so the call still returns exact labels.
    // Range and offset errors found before the timeout are reported instead.
    if ((status_host[0] & kErrBarrierBit) && !(status_host[0] & (kErrRangeBit | kErrOffsetsBit)) && refused) {
        *refused = true;
        return CC_OK;
    }
    if (status_host[0] == 0 && status_host[kStatusDeep]) return finish_deep(h, pb, status_host, s);
    return CC_OK;
}

// Fallback without a persistent grid: the batch as one graph on vert_off[G]
// vertices (graph g's ids shifted by vert_off[g]), labelled by the single-graph
// SV loop (R1), then shifted back to graph-local labels.  Same labels, one
// host round trip per pass.
static int run_union(Workspace& ws, const BatchArgsHost& h, hipStream_t s, unsigned long long* host,
                     cc_batch_stats* stats) {
    const int64_t m = h.m, n = h.n;
    const size_t half = ((size_t)m * sizeof(int32_t) + 255) & ~(size_t)255;
    void *pg, *pf;
    int rc;
    if ((rc = ws.get(WS_ADJ, 2 * half + 256, &pg))) return rc;
    if ((rc = ws.get(WS_HISTOUT, 64, &pf))) return rc;
    int32_t* gu = (int32_t*)pg;
    int32_t* gv = (int32_t*)((char*)pg + half);
    unsigned long long* bad = (unsigned long long*)pf;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
    }
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) e = launch_union_relabel(h.u, h.v, h.edge_off, h.vert_off, h.G, m, gu, gv, bad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "union relabel");
    else if (host[0]) rc = fail(CC_EINVAL, "edge_off / vert_off are not non-decreasing");
    cc_stats st;
    memset(&st, 0, sizeof st);
    if (rc == CC_OK) {
        Call c;
        c.ws = &ws;
        c.stream = s;
        c.u = gu;
        c.v = gv;
        c.m = m;
        c.n = (int32_t)n;
        c.parent = h.labels;
        cc_default_options(&c.opt);
        c.stats = &st;
        Timer tm(false, s);
        c.timer = &tm;
        e = launch_sv_init(h.labels, (int32_t)n, s);
        if (e != hipSuccess) rc = hip_fail(e, "sv_init launch");
        if (rc == CC_OK && m > 0) {
            SvInput in;
            in.soa = true;
            in.u = gu;
            in.v = gv;
            in.m = m;
            rc = run_sv(c, in, CC_R1_SV, 8.0, 0);
            if (rc == CC_ERANGE) rc = fail(CC_ERANGE, "edges have an endpoint outside their graph's [0, n_g)");
        }
        if (rc == CC_OK && (e = launch_union_unshift(h.labels, h.vert_off, h.G, n, s)) != hipSuccess)
            rc = hip_fail(e, "union unshift");
    }
    if (rc == CC_OK && stats) {
        float t = 0.f;
        if ((e = hipEventRecord(e1, s)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess)
            (void)hipEventElapsedTime(&t, e0, e1);
        stats->passes = st.sv_passes;
        stats->blocks = 0;   // no persistent grid
        stats->max_link = 1;
        stats->tile_edges = 0;
        stats->total_edges = m;
        stats->total_vertices = n;
        stats->ms_total = t;
        stats->atomics = st.sv_atomics;
        stats->chase_reads = st.sv_chase_reads;
        for (int i = 0; i < std::min(st.sv_passes, 64); ++i) {
            stats->edges_read += st.active_edges[i];
            if (i > 0) stats->survivors_written += st.active_edges[i];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == CC_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    return rc;
}

static int status_code(const unsigned long long* st) {
    if (st[0] & 1) return fail(CC_ERANGE, "%llu edges have an endpoint outside their graph's [0, n_g)", st[2]);
    if (st[0] & 2) return fail(CC_EINVAL, "edge_off / vert_off are not non-decreasing");
    if (st[0] & 4) return fail(CC_EINTERNAL, "grid barrier timed out");   // only without a fallback
    if (st[0] & 8) return fail(CC_EINTERNAL, "pass cap reached");
    if (st[0] & 16) return fail(CC_EINTERNAL, "flatten did not finish");
    return CC_OK;
}

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_label_batched_ex(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                               int32_t G, int32_t* labels, void* stream, int32_t tile_edges, int32_t max_link,
                               cc_batch_stats* stats) {
    if (stats) memset(stats, 0, sizeof *stats);
    if (G < 0) return fail(CC_EINVAL, "negative G");
    if (tile_edges < 0 || max_link < 0) return fail(CC_EINVAL, "negative tile_edges / max_link");
    if (G == 0) return CC_OK;
    if (!edge_off || !vert_off) return fail(CC_EINVAL, "NULL offsets");
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::lock_guard<std::mutex> guard(ws->mu);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* host;
    if ((rc = ws->pinned((void**)&host))) return rc;
    int64_t* h64 = (int64_t*)host;
    hipError_t e = hipMemcpyAsync(h64, edge_off, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h64 + 1, edge_off + G, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h64 + 2, vert_off, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h64 + 3, vert_off + G, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "offset readback");
    const int64_t m = h64[1], n = h64[3];
    if (h64[0] != 0 || h64[2] != 0) return fail(CC_EINVAL, "edge_off[0] and vert_off[0] must be 0");
    if (m < 0 || n < 0 || n > INT32_MAX) return fail(CC_EINVAL, "bad totals (m=%lld, n=%lld)", (long long)m, (long long)n);
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge arrays");
    if (n > 0 && !labels) return fail(CC_EINVAL, "NULL labels");
    if (m > 0 && n == 0) return fail(CC_ERANGE, "edges given for graphs without vertices");
    if (m > (int64_t)2048 * INT32_MAX) return fail(CC_EINVAL, "too many edges");
    int maxb = 0;
    if ((e = batched_max_blocks(&maxb)) != hipSuccess) return hip_fail(e, "occupancy query");
    if (maxb < 1) return fail(CC_EINTERNAL, "persistent kernel does not fit on this device");
    BatchArgsHost h{};
    h.u = u;
    h.v = v;
    h.edge_off = edge_off;
    h.vert_off = vert_off;
    h.G = G;
    h.m = m;
    h.n = (int32_t)n;
    h.labels = labels;
    h.max_passes = 100000;
    h.barrier_ticks = barrier_ticks();
    Tuned cfg;
    maxb &= ~7;   // the tile walk gives each of the 8 XCDs the same number of workgroups
    if (maxb < 8) return fail(CC_EINTERNAL, "persistent grid too small for this device");
    std::vector<int> bcand, lcand;
    if (tile_edges > 0) {
        int64_t b = (m + tile_edges - 1) / tile_edges;
        b = std::max<int64_t>(8, std::min<int64_t>(b, maxb));
        bcand.push_back((int)(b & ~(int64_t)7));
    } else {
        for (int cb : {256, 512, 1024})
            if (std::min(cb, maxb) != (bcand.empty() ? -1 : bcand.back())) bcand.push_back(std::min(cb, maxb));
    }
    if (max_link > 0) lcand.push_back(max_link);
    else lcand = {1, 4};
    if (bcand.size() == 1 && lcand.size() == 1) {
        cfg = Tuned{bcand[0], lcand[0]};
    } else {
        const bool cacheable = tile_edges == 0 && max_link == 0;
        std::string key = tune_key(ws->device, m, (int32_t)n, G);
        if (cacheable) {
            std::lock_guard<std::mutex> g(g_tune_mu);
            tune_load();
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                cfg = it->second;
                cfg.blocks = std::max(8, std::min(cfg.blocks, maxb) & ~7);
            }
        }
        if (cfg.blocks <= 0) {
            // time every candidate on this input (each computes the same labels)
            double best = 1e300;
            for (int b : bcand)
                for (int l : lcand) {
                    double ms = 0;
                    bool refused = false;
                    if ((rc = run_once(*ws, h, b, l, s, host, &ms, &refused))) return rc;
                    if (refused) return run_union(*ws, h, s, host, stats);
                    if ((rc = status_code(host))) return rc;
                    if (ms < best) {
                        best = ms;
                        cfg = Tuned{b, l};
                    }
                }
            if (cacheable) {
                std::lock_guard<std::mutex> g(g_tune_mu);
                tune_store(key, cfg);
            }
        }
    }
    double ms = 0;
    bool refused = false;
    if ((rc = run_once(*ws, h, cfg.blocks, cfg.link, s, host, stats ? &ms : nullptr, &refused))) return rc;
    if (refused) return run_union(*ws, h, s, host, stats);
    if ((rc = status_code(host))) return rc;
    if (stats) {
        const int passes = (int)host[1];
        stats->passes = passes;
        stats->blocks = cfg.blocks;
        stats->max_link = cfg.link;
        stats->tile_edges = (int32_t)std::min<int64_t>(INT32_MAX, m > 0 ? (m + cfg.blocks - 1) / cfg.blocks : 0);
        stats->total_edges = m;
        stats->total_vertices = n;
        stats->ms_total = ms;
        const unsigned long long* bs = host + kBstatHost;
        const int nbk = cfg.blocks;
        for (int i = 0; i < nbk; ++i) {
            stats->atomics += (int64_t)bs[i];
            stats->chase_reads += (int64_t)bs[nbk + i];
            stats->edges_read += (int64_t)bs[2 * nbk + i];
            stats->survivors_written += (int64_t)bs[3 * nbk + i];
        }
        // barrier stamps (100 MHz wall clock): pass i runs between stamps i and i+1
        for (int i = 0; i < 32 && i + 1 < 40 && i < passes + 1; ++i) {
            const unsigned long long a = host[8 + i], b = host[8 + i + 1];
            stats->pass_ms[i] = (b > a) ? (float)((double)(b - a) * 1e-5) : 0.f;
        }
    }
    return CC_OK;
}

CC_API int cc_label_batched(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                            int32_t G, int32_t* labels, void* stream) {
    return cc_label_batched_ex(u, v, edge_off, vert_off, G, labels, stream, 0, 0, nullptr);
}
