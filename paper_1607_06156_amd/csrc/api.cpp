// C ABI of libccmi: validation, workspace, route choice and the host loops
// that drive the HIP kernels.  See include/cc.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/cc.h"
#include "common.hpp"
#include "hubs.hpp"
#include "internal.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}


int hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return fail(CC_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(CC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------- failure injection
static std::atomic<int64_t> g_fail_alloc{0};
static std::once_flag g_fail_alloc_env;

bool alloc_fault() {
    // CCMI_FAIL_ALLOC=k in the environment arms the countdown once, at the
    // process's first allocation check
    std::call_once(g_fail_alloc_env, [] {
        const char* e = getenv("CCMI_FAIL_ALLOC");
        const long long k = e ? atoll(e) : 0;
        if (k > 0) g_fail_alloc.store((int64_t)k);
    });
    int64_t k = g_fail_alloc.load();
    while (k > 0)
        if (g_fail_alloc.compare_exchange_weak(k, k - 1)) return k == 1;
    return false;
}

// --------------------------------------------------------------- workspace
// Shared pool of pinned staging buffers for the calls that do not use the
// device's cached workspace: a call leases one and returns it at its end, so
// calls running at once on different streams never share a buffer.
static std::mutex g_stage_mu;
static std::vector<void*> g_stage_free;   // idle buffers
static std::vector<void*> g_stage_all;    // every buffer made (freed by cc_shutdown)

static int lease_stage(void** out) {
    {
        std::lock_guard<std::mutex> g(g_stage_mu);
        if (!g_stage_free.empty()) {
            *out = g_stage_free.back();
            g_stage_free.pop_back();
            return CC_OK;
        }
    }
    void* p = nullptr;
    hipError_t e = alloc_fault() ? hipErrorOutOfMemory : hipHostMalloc(&p, Workspace::kHostBytes, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    std::lock_guard<std::mutex> g(g_stage_mu);
    g_stage_all.push_back(p);
    *out = p;
    return CC_OK;
}

static void return_stage(void* p) {
    std::lock_guard<std::mutex> g(g_stage_mu);
    g_stage_free.push_back(p);
}

Workspace::~Workspace() {
    if (mode == kCached) release();
    else finish();
}

void Workspace::release() {
    for (auto& b : bufs) {
        if (b.ptr) (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (host && !host_external && !host_leased) (void)hipHostFree(host);
    host = nullptr;
}

void Workspace::finish() {
    if (mode == kPool) {
        for (auto& b : bufs) {
            if (b.ptr) (void)hipFreeAsync(b.ptr, stream);
            b.ptr = nullptr;
            b.bytes = 0;
        }
    }
    if (host_leased && host) return_stage(host);
    if (host_leased) host = nullptr;
    host_leased = false;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int Workspace::get(int slot, size_t bytes, void** out) {
    if (bytes == 0) bytes = 256;
    Buf& b = bufs[slot];
    if (b.bytes >= bytes) {
        *out = b.ptr;
        return CC_OK;
    }
    if (mode == kArena) {
        // first use: the slot's whole bound; a request beyond it (none is
        // expected) gets a fresh region if the block still has room
        const size_t want = align256(std::max(bytes, b.ptr ? bytes : bound[slot]));
        const size_t base = align256((size_t)(uintptr_t)arena) - (size_t)(uintptr_t)arena;
        if (base + arena_used + want > arena_bytes)
            return fail(CC_ENOMEM, "workspace of %zu bytes is too small for this call (slot %d needs %zu more)",
                        arena_bytes, slot, want);
        b.ptr = arena + base + arena_used;
        b.bytes = want;
        arena_used += want;
        *out = b.ptr;
        return CC_OK;
    }
    if (mode == kPool) {
        if (b.ptr) {
            hipError_t e = hipFreeAsync(b.ptr, stream);
            b.ptr = nullptr;
            b.bytes = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFreeAsync(workspace)");
        }
        hipError_t e = alloc_fault() ? hipErrorOutOfMemory : hipMallocFromPoolAsync(&b.ptr, bytes, pool, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.ptr = nullptr;
            return hip_fail(e, "hipMallocFromPoolAsync(workspace)");
        }
        b.bytes = bytes;
        *out = b.ptr;
        return CC_OK;
    }
    if (b.ptr) {
        hipError_t e = hipFree(b.ptr);
        if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;  // headroom against repeated growth
    hipError_t e = alloc_fault() ? hipErrorOutOfMemory : hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return hip_fail(e, "hipMalloc(workspace)");
    }
    b.bytes = want;
    *out = b.ptr;
    return CC_OK;
}

int Workspace::pinned(void** out) {
    if (!host) {
        if (mode == kCached) {
            hipError_t e = alloc_fault() ? hipErrorOutOfMemory : hipHostMalloc(&host, kHostBytes, hipHostMallocDefault);
            if (e != hipSuccess) {
                host = nullptr;
                return hip_fail(e, "hipHostMalloc");
            }
        } else {
            int rc = lease_stage(&host);
            if (rc) return rc;
            host_leased = true;
        }
    }
    *out = host;
    return CC_OK;
}

static std::mutex g_ws_mu;
static std::unordered_map<int, Workspace*> g_ws;

// One more stream per device (default priority, not synchronising with the
// null stream): the power-law fit runs on it beside a speculative SV launch.
static std::mutex g_side_mu;
static std::unordered_map<int, hipStream_t> g_side;

int side_stream(hipStream_t* out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_side_mu);
    auto it = g_side.find(dev);
    if (it == g_side.end()) {
        hipStream_t s = nullptr;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        it = g_side.emplace(dev, s).first;
    }
    *out = it->second;
    return CC_OK;
}
static std::unordered_map<int, hipMemPool_t> g_pools;

int acquire_workspace(Workspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto it = g_ws.find(dev);
    if (it == g_ws.end()) it = g_ws.emplace(dev, new Workspace()).first;
    it->second->device = dev;
    *out = it->second;
    return CC_OK;
}

// The library's memory pool on the current device: stream-ordered
// allocations that it keeps after they are freed (release threshold at its
// maximum), so a call of the same size as an earlier one maps no new memory.
// cc_release_workspace trims it.
int pool_workspace(Workspace* ws, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto it = g_pools.find(dev);
    if (it == g_pools.end()) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof props);
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return hip_fail(e, "hipMemPoolCreate");
        uint64_t keep = UINT64_MAX;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return hip_fail(e, "hipMemPoolSetAttribute");
        }
        it = g_pools.emplace(dev, pool).first;
    }
    ws->mode = Workspace::kPool;
    ws->device = dev;
    ws->stream = s;
    ws->pool = it->second;
    return CC_OK;
}

size_t workspace_bound(int64_t m, int32_t n, bool sv_only, size_t* per_slot) {
    size_t b[WS_NSLOTS] = {};
    const size_t M = (size_t)std::max<int64_t>(m, 0), N = (size_t)std::max<int32_t>(n, 0);
    // SV: at most 8 chunks of 2048 segments, each segment ceil(m / nseg)
    // slots, so the slots number fewer than m + 16384; the BFS route's rest
    // (from the CSR rows or the filtered list) holds at most m edges
    const size_t slots = M + 8 * 2048;
    b[WS_EDGES0] = slots * 8;
    b[WS_EDGES1] = slots * 8;
    b[WS_HOOKED] = slots * 4;
    b[WS_SEGCOUNT] = (size_t)8 * 2048 * 7 * sizeof(uint32_t);
    b[WS_TOTALS] = 64 * sizeof(unsigned long long);
    if (M >= ((size_t)1 << 22)) b[WS_GIANT] = ((N + 63) / 64) * 8;   // a chunked first pass (pass0_chunks)
    if (!sv_only) {
        BucketPlan p;
        if (bucket_plan(n, m, &p) == 0 && m < ((int64_t)1 << 31)) {
            const size_t counts = align256((size_t)p.nblk * p.B * sizeof(uint32_t));
            b[WS_HIST] = counts + (size_t)(2 * p.B + 3) * sizeof(unsigned long long) +
                         (size_t)p.B * kGroups * sizeof(uint32_t);
            b[WS_CURSOR] = 16 * M;   // two-level scatter with the other ends, CSR regroup, the rest's arrays
            b[WS_QUEUE] = align256(2 * M * sizeof(uint16_t)) + 2 * M * sizeof(int32_t);
            b[WS_DEG] = 4 * N;
            if (b[WS_GIANT]) b[WS_GIANT] = align256(b[WS_GIANT]) + kHubBytes;   // the hub arrays
            const size_t tail = std::min(N, 2 * M / kExactBins + 1);
            b[WS_TAIL] = 4 * tail;
            b[WS_HISTOUT] = (64 + kExactBins + 4) * sizeof(unsigned long long);
            b[WS_OFF] = 8 * (N + 1);
            b[WS_ADJ] = 8 * M;
            b[WS_BITS] = 12 * ((N + 31) / 32);
            b[WS_MLP] = 512;
            // fit: per distinct degree 3 doubles in, and per candidate an
            // index and 2 doubles out
            const size_t V = kExactBins + tail;
            b[WS_KS] = 44 * V + 64;
            // BFS queues and prefix sums share the SV slots
            b[WS_HOOKED] = std::max(b[WS_HOOKED], 8 * N);
            b[WS_SEGCOUNT] = std::max(b[WS_SEGCOUNT], 8 * (N + N / 1024 + 8));
        }
    }
    size_t total = 256;
    for (int i = 0; i < WS_NSLOTS; ++i) {
        if (per_slot) per_slot[i] = b[i];
        if (b[i]) total += align256(b[i]);
    }
    return total;
}

// ------------------------------------------------------------------ timing
hipError_t create_timing_event(hipEvent_t* ev) { return hipEventCreateWithFlags(ev, hipEventDisableSystemFence); }

Timer::Timer(bool on, hipStream_t s) : enabled(on), stream(s) {}
Timer::~Timer() {
    for (auto ev : events) (void)hipEventDestroy(ev);
}
int Timer::mark() {
    if (!enabled) return -1;
    hipEvent_t ev;
    if (create_timing_event(&ev) != hipSuccess) return -1;
    (void)hipEventRecord(ev, stream);
    events.push_back(ev);
    return (int)events.size() - 1;
}
double Timer::ms(int a, int b) {
    if (!enabled || a < 0 || b < 0) return 0.0;
    (void)hipEventSynchronize(events[b]);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, events[a], events[b]);
    return (double)t;
}

// ---------------------------------------------------------------- SV loop
int choose_nseg(int64_t m) {
    int64_t s = (m + 1023) / 1024;
    if (s < 1) s = 1;
    if (s > 2048) s = 2048;
    return (int)s;
}

// hooked roots are pointer-jumped after a pass only if at most this many per survivor
constexpr int64_t kLazyJump = 8;
// The first chunk of the first pass, where the trees grow from single
// vertices, runs as two launches with a full flatten between them when the
// graph has at least kSplitDegree edges per vertex (a flatten costs O(n); on
// sparse graphs it costs more than the shorter finds save): first a small
// one over 1/kFirstLaunch of its segments, then the rest.  Nearly every edge
// of that first launch hooks, many of them onto the same few hub roots, and
// same-address device atomics serialise: the fewer workgroups in flight, the
// shorter those queues.  Measured on MI355X (forced SV, R-MAT scale 24 /
// noisy R-MAT scale 24): one launch 9.0 / 10.7 ms; halves 9.2 / 9.6 ms;
// first 1/4: 9.1 / 8.4 ms; first 1/8: 8.6 / 7.8 ms; first 1/16: 8.8 / 8.2 ms;
// giving each half its own 2048 workgroups (more in flight) made the first
// launch 2.5x slower.
constexpr int kFirstLaunch = 8;
constexpr int64_t kSplitDegree = 8;
// On lists with more than kMergeAfter + 2 first-pass chunks, chunks
// kMergeAfter and later run as one launch.  Measured on MI355X (forced SV,
// each chunk its own launch / from the third chunk on as one / from the
// fourth): R-MAT scale 24 3.98 / 3.65 / 3.70 ms, noisy R-MAT 3.92 / 3.49 /
// 3.55 ms; the 8192^2 lattice (4 chunks) 10.08 / 11.04 ms when merged from
// the third, the 200 M-vertex forest (4 chunks) 22.2 / 20.7 ms.
constexpr int kMergeAfter = 2;

// Chunks of the first pass.  Within one pass the trees only grow (no
// shortcut runs while hooks are in flight), so the finds of late edges walk
// long chains.  Cutting the first pass into chunks with a full pointer-jumping
// shortcut after each keeps the trees flat; the shortcut costs O(n), so the
// chunk count follows m / n.  Short lists take one chunk: there the extra
// launches would cost more than the links they save.
int pass0_chunks(int64_t m, int32_t n) {
    if (n <= 0 || m < ((int64_t)1 << 22)) return 1;
    int64_t k = (5 * m + 2 * (int64_t)n - 1) / (2 * (int64_t)n);   // ceil(2.5 m / n)
    if (k < 1) k = 1;
    if (k > 8) k = 8;
    return (int)k;
}

// Flatten rounds until every vertex points at its root.  A round leaves *open
// set when some root lay more than kMaxHops links up; each round divides the
// depth of the forest by at least kMaxHops, so a forest of depth below n takes
// at most log(n) / log(kMaxHops) + 1 rounds.  *extra counts the rounds after
// the first.  hpin: pinned host word.
constexpr int kMaxFlattenRounds = 16;
static int flatten_all(Call& c, unsigned long long* open, unsigned long long* hpin, int* extra) {
    for (int r = 0;; ++r) {
        hipError_t e = hipSuccess;
        if (r > 0) e = hipMemsetAsync(open, 0, sizeof(*open), c.stream);   // round 0 starts clear
        int k0 = c.kbeg();
        if (e == hipSuccess) e = launch_sv_finalize(c.parent, c.n, open, c.stream);
        if (e != hipSuccess) return hip_fail(e, "sv_finalize launch");
        c.kend(CC_K_SV_FINALIZE, k0, 8.0 * c.n);
        if (c.stats) c.bytes += 8.0 * c.n;
        e = hipMemcpyAsync(hpin, open, sizeof(*open), hipMemcpyDeviceToHost, c.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return hip_fail(e, "flatten readback");
        if (!*hpin) return CC_OK;
        ++*extra;
        if (r + 1 >= kMaxFlattenRounds) return fail(CC_EINTERNAL, "flatten did not finish in %d rounds", r + 1);
    }
}

// Segments of the first pass over a caller's list of m0 edges: chunks of
// nseg_chunk segments of cap edges; on dense lists the first chunk runs as
// [0, cut) and [cut, nseg_chunk) (split = 2).
struct SvGeom {
    int chunks = 1, nseg_chunk = 0, nseg = 0, split = 1, cut = 1;
    int64_t cap = 1;
};

static SvGeom sv_geometry(int64_t m0, int32_t n) {
    SvGeom g;
    g.chunks = pass0_chunks(m0, n);
    g.nseg_chunk = choose_nseg((m0 + g.chunks - 1) / g.chunks);
    g.nseg = g.chunks * g.nseg_chunk;
    g.cap = (m0 + g.nseg - 1) / g.nseg;
    if (g.cap < 1) g.cap = 1;
    g.split = g.chunks > 1 && m0 >= kSplitDegree * (int64_t)n && g.nseg_chunk >= 2 ? 2 : 1;
    g.cut = std::max(1, g.nseg_chunk / kFirstLaunch);
    return g;
}

// The first launch of the first pass, enqueued before the route is known
// (while the host fits the degree distribution).  Only on lists cut into
// several chunks; run_sv(..., spec) then goes on from it.  It needs no
// result of the degree pass: every id is range-checked by the pass itself.
int sv_speculate(Call& c, const SvInput& in0, SvSpec* spec) {
    spec->launched = false;
    if (!in0.soa || in0.m <= 0) return CC_OK;
    const SvGeom g = sv_geometry(in0.m, c.n);
    if (g.chunks <= 1) return CC_OK;
    Workspace& ws = *c.ws;
    const size_t slots = (size_t)g.nseg * (size_t)g.cap;
    void *pbuf0, *phook, *pcnt, *ptot;
    int rc;
    if ((rc = ws.get(WS_EDGES0, slots * sizeof(int2), &pbuf0))) return rc;
    if ((rc = ws.get(WS_HOOKED, slots * sizeof(int32_t), &phook))) return rc;
    if ((rc = ws.get(WS_SEGCOUNT, (size_t)g.nseg * 7 * sizeof(uint32_t), &pcnt))) return rc;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &ptot))) return rc;
    unsigned long long* totals = (unsigned long long*)ptot;
    hipError_t e = hipMemsetAsync(totals, 0, 64 * sizeof(unsigned long long), c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    // the same arrays and launch as run_sv's first: survivors to segment
    // buffer 0 with counts in array 1, hooks counted in array 3
    const int s1 = g.split == 2 ? g.cut : g.nseg_chunk;
    SegList out{(int2*)pbuf0, g.cap, g.nseg, (uint32_t*)pcnt + (size_t)1 * g.nseg};
    spec->t0 = c.timer->mark();
    int k0 = c.kbeg();
    e = launch_sv_pass_soa(in0.u, in0.v, in0.m, c.n, c.parent, out, 0, s1, 1, 1, (int32_t*)phook,
                           (uint32_t*)pcnt + (size_t)3 * g.nseg, totals, (uint32_t*)pcnt + (size_t)4 * g.nseg, nullptr,
                           nullptr, c.stream);
    if (e != hipSuccess) return hip_fail(e, "sv_pass launch");
    spec->rec = c.kend(CC_K_SV_PASS, k0, 16.0 * (double)std::min<int64_t>(in0.m, (int64_t)s1 * g.cap));
    spec->t1 = c.timer->mark();
    spec->launched = true;
    return CC_OK;
}

int run_sv(Call& c, const SvInput& in0, int policy, double theta, int max_passes, const SvSpec* spec) {
    Workspace& ws = *c.ws;
    const int64_t m0 = in0.soa ? in0.m : 0;
    const bool resume = spec && spec->launched && in0.soa;
    int nseg;
    int64_t cap;
    int chunks = 1, nseg_chunk = 0;
    SvGeom geom;
    if (in0.soa) {
        geom = sv_geometry(m0, c.n);
        chunks = geom.chunks;
        nseg_chunk = geom.nseg_chunk;
        nseg = geom.nseg;
        cap = geom.cap;
    } else {
        nseg = in0.seg.nseg;
        cap = in0.seg.cap;
    }
    const size_t slots = (size_t)nseg * (size_t)cap;
    void *pbuf0, *pbuf1, *phook, *pcnt;
    int rc;
    // the input segment list (if any) already lives in WS_EDGES0; survivors go
    // to the other buffer
    if ((rc = ws.get(WS_EDGES0, slots * sizeof(int2), &pbuf0))) return rc;
    if ((rc = ws.get(WS_EDGES1, slots * sizeof(int2), &pbuf1))) return rc;
    if ((rc = ws.get(WS_HOOKED, slots * sizeof(int32_t), &phook))) return rc;
    // per segment: 3 rotating survivor counts, the hook count, 3 statistics
    if ((rc = ws.get(WS_SEGCOUNT, (size_t)nseg * 7 * sizeof(uint32_t), &pcnt))) return rc;
    void* ptot;
    if ((rc = ws.get(WS_TOTALS, 64 * sizeof(unsigned long long), &ptot))) return rc;
    unsigned long long* totals = (unsigned long long*)ptot;
    unsigned long long* htot;
    if ((rc = ws.pinned((void**)&htot))) return rc;
    uint32_t* cnt[4];
    for (int i = 0; i < 4; ++i) cnt[i] = (uint32_t*)pcnt + (size_t)i * nseg;
    uint32_t* hooked_count = cnt[3];
    uint32_t* segstat = (uint32_t*)pcnt + (size_t)4 * nseg;
    // The largest tree during a chunked first pass (see below): its root in
    // an int32 word of the totals block, its membership bitmap in WS_GIANT.
    int32_t* gflag = (int32_t*)(totals + 10);
    uint32_t* gbits = nullptr;
    // With the degrees known, the hubs' list, their table and the table of
    // those in the largest tree follow the bitmap; their count is a word of
    // the totals block.
    int32_t* hub_list = nullptr;
    int4 *hub_ids = nullptr, *hub_tree = nullptr;
    uint32_t* hub_count = (uint32_t*)(totals + 11);
    bool hubs_listed = false;
    if (in0.soa && chunks > 1) {
        const size_t bits_bytes = (size_t)((c.n + 63) / 64) * 8;
        const bool hubs = c.hub_deg && c.hub_min > 0;
        void* pg;
        if ((rc = ws.get(WS_GIANT, hubs ? align256(bits_bytes) + kHubBytes : bits_bytes, &pg))) return rc;
        gbits = (uint32_t*)pg;
        if (hubs) {
            hub_list = (int32_t*)((char*)pg + align256(bits_bytes));
            hub_ids = (int4*)(hub_list + kHubMax);
            hub_tree = hub_ids + kHubBuckets;
        }
    }
    int2* bufs[2] = {(int2*)pbuf0, (int2*)pbuf1};

    // (resuming after sv_speculate: its launch's counters are already in totals)
    hipError_t e = resume ? hipSuccess : hipMemsetAsync(totals, 0, 64 * sizeof(unsigned long long), c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");

    bool in_soa = in0.soa;
    SegList in{nullptr, cap, nseg, nullptr};
    int in_buf = 0, in_cnt = 0;
    int deep_rounds = 0;   // flatten rounds forced by deep chains
    if (!in_soa) {
        // caller placed the list in WS_EDGES0 with counts in cnt[0]
        if (in0.seg.buf != bufs[0]) return fail(CC_EINTERNAL, "segment list not in workspace");
        hipError_t ce = hipMemcpyAsync(cnt[0], in0.seg.count, (size_t)nseg * sizeof(uint32_t),
                                       hipMemcpyDeviceToDevice, c.stream);
        if (ce != hipSuccess) return hip_fail(ce, "hipMemcpyAsync(counts)");
        in = SegList{bufs[0], cap, nseg, cnt[0]};
    }
    int64_t m_in = in0.soa ? m0 : in0.m;
    // R1: one hook attempt per edge per pass (the paper's one join per
    // iteration); R2: up to theta attempts, following the links it meets
    const int max_link = policy == CC_R2_SV_THETA ? (int)std::min(theta, 1e9) : 1;
    int pass = 0;
    while (m_in > 0) {
        if (max_passes > 0 && pass >= max_passes)
            return fail(CC_EINTERNAL, "SV did not converge within %d passes", max_passes);
        const bool write = true;
        const int out_buf = in_soa ? 0 : 1 - in_buf;
        // out counts: any array other than the input's and the hooks'
        int out_cnt = (in_cnt + 1) % 3;
        SegList out{bufs[out_buf], cap, nseg, cnt[out_cnt]};
        int rec_pass = -1;
        double flat_bytes = 0.0;
        int64_t filt_edges = 0;   // edges of this pass read by launches with the bitmap
        int last_lo = 0;          // first segment of the first pass's last launch
        if (in_soa) {
            // chunk k covers segments [k * nseg_chunk, (k + 1) * nseg_chunk);
            // on dense graphs the first chunk is launched as [0, cut), [cut, nseg_chunk)
            const int split = geom.split;
            const int cut = geom.cut;
            // On dense lists (more than kMergeAfter + 2 chunks) the chunks from
            // kMergeAfter on run as one launch: by then the largest tree's
            // bitmap drops nearly all of their edges, and the flattens, picks
            // and bitmaps between them cost more than the shallower trees
            // save.  Sparse lists keep every chunk (a lattice's largest tree
            // appears only in its last chunks).
            const int merge_at = chunks > kMergeAfter + 2 ? kMergeAfter : chunks;
            last_lo = std::min(merge_at, chunks - 1) * nseg_chunk;
            int chain = -1;   // end mark of the previous group of launches
            for (int k = 0; k < chunks; ++k) {
                for (int part = 0; part < (k == 0 ? split : 1); ++part) {
                    const int s0 = k > 0 ? k * nseg_chunk : (part == 0 ? 0 : cut);
                    const int s1 = k >= merge_at ? chunks * nseg_chunk
                                 : k > 0 ? (k + 1) * nseg_chunk : (split == 1 || part == 1 ? nseg_chunk : cut);
                    const bool filt = s0 > 0 && gbits;
                    if (resume && pass == 0 && k == 0 && part == 0) {
                        // this launch was enqueued by sv_speculate, with the same
                        // segments, arrays and hook rule (R2's later attempts only
                        // add hooks, so its first launch may use R1's)
                        rec_pass = spec->rec;
                        chain = -1;   // the fit's kernels and copies ran after it
                        continue;
                    }
                    if (s0 > 0) {
                        int kf = c.kbeg_after(chain);
                        e = launch_sv_finalize(c.parent, c.n, totals + 6, c.stream);
                        if (e != hipSuccess) return hip_fail(e, "sv_finalize launch");
                        // parent read + one gather per vertex, at most one write
                        chain = c.kmark(c.kend(CC_K_SV_SHORTCUT, kf, 12.0 * c.n));
                        flat_bytes += 12.0 * c.n;
                    }
                    if (filt) {
                        // Edges inside the largest tree are finished (Section
                        // III-A.4); after the flatten, a bitmap of that tree
                        // lets the next launch drop them with two bit probes
                        // instead of two gathers of parent[].  Sampled roots
                        // pick the tree; none holding 1/16 of the samples
                        // turns the probes off.
                        int kg = c.kbeg_after(chain);
                        double gbytes = 4.0 * c.n + c.n / 8.0;   // parent read per vertex, bitmap written
                        e = hipSuccess;
                        if (hub_list && !hubs_listed) {
                            // once per call: the hubs (degree read per vertex) and their table
                            e = launch_hub_list(c.hub_deg, c.n, c.hub_min, hub_list, hub_count, hub_ids, c.stream);
                            hubs_listed = true;
                            gbytes += 4.0 * c.n;
                        }
                        if (e == hipSuccess) e = launch_giant_pick(c.parent, c.n, gflag, c.stream);
                        if (e == hipSuccess)
                            e = hub_list ? launch_giant_bits_hubs(c.parent, c.n, gflag, gbits, hub_ids, hub_tree,
                                                                  c.stream)
                                         : launch_giant_bits(c.parent, c.n, gflag, gbits, c.stream);
                        if (e != hipSuccess) return hip_fail(e, "giant bitmap launch");
                        chain = c.kmark(c.kend(CC_K_SV_SHORTCUT, kg, gbytes));
                        flat_bytes += gbytes;
                    }
                    int k0 = c.kbeg_after(chain);
                    e = launch_sv_pass_soa_hubs(in0.u, in0.v, m0, c.n, c.parent, out, s0, s1 - s0, write ? 1 : 0,
                                                max_link, (int32_t*)phook, hooked_count, totals, segstat,
                                                filt ? gbits : nullptr, filt ? gflag : nullptr,
                                                filt ? hub_tree : nullptr, c.stream);
                    if (e != hipSuccess) return hip_fail(e, "sv_pass launch");
                    // this launch's edges (read + two 4-byte gathers or bit
                    // probes each); the rest of the pass's bytes go to the
                    // last launch below
                    const int64_t e0 = std::min<int64_t>(m0, (int64_t)s0 * cap);
                    const int64_t e1 = std::min<int64_t>(m0, (int64_t)s1 * cap);
                    rec_pass = c.kend(CC_K_SV_PASS, k0, 16.0 * (double)(e1 - e0));
                    chain = c.kmark(rec_pass);
                    if (filt) filt_edges += e1 - e0;
                }
                if (k >= merge_at) break;
            }
        } else {
            // a long list handed over by an earlier step (the edges a BFS left)
            // gets the same chunked first pass as the caller's list
            const int segchunks = pass == 0 ? pass0_chunks(m_in, c.n) : 1;
            const int per = (nseg + segchunks - 1) / segchunks;
            int chain = -1;   // end mark of the previous group of launches
            for (int s0 = 0; s0 < nseg; s0 += per) {
                if (s0 > 0) {
                    int kf = c.kbeg_after(chain);
                    e = launch_sv_finalize(c.parent, c.n, totals + 6, c.stream);
                    if (e != hipSuccess) return hip_fail(e, "sv_finalize launch");
                    chain = c.kmark(c.kend(CC_K_SV_SHORTCUT, kf, 12.0 * c.n));
                    flat_bytes += 12.0 * c.n;
                }
                const int nb = std::min(per, nseg - s0);
                int k0 = c.kbeg_after(chain);
                e = launch_sv_pass_seg(in, s0, nb, c.parent, out, write ? 1 : 0, max_link, (int32_t*)phook,
                                       hooked_count, totals, segstat, c.stream);
                if (e != hipSuccess) return hip_fail(e, "sv_pass launch");
                // this chunk's share of the edges (segments hold about equal counts)
                rec_pass = c.kend(CC_K_SV_PASS, k0, 16.0 * (double)m_in * nb / nseg);
                chain = c.kmark(rec_pass);
            }
        }
        // After a chunked first pass, the full flatten before each launch has
        // already jumped every root hooked before the last launch: only its
        // segments hold roots still to jump.
        const int jump_lo = in_soa && chunks > 1 ? last_lo : 0;
        e = launch_sv_totals(hooked_count, out.count, nseg, jump_lo, segstat, totals, c.stream);
        if (e != hipSuccess) return hip_fail(e, "sv_totals launch");
        e = hipMemcpyAsync(htot, totals, 12 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c.stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(totals)");
        e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        if (htot[2]) return fail(CC_ERANGE, "%llu edge endpoints outside [0, n)", (unsigned long long)htot[2]);
        const int64_t kept = (int64_t)htot[0];
        const int64_t hooks = (int64_t)htot[1];
        const int64_t fresh = (int64_t)htot[3];   // hooked since the last full flatten
        // the byte model's counts, read before a deep flatten reuses htot[8]
        const int64_t natom = (int64_t)htot[7], nchase = (int64_t)htot[8], ndrop = (int64_t)htot[9];
        // Finds that stopped at the hop bound: the pass left deep chains, so
        // the forest is flattened completely before the next pass.
        const bool deep = kept > 0 && htot[4] > 0;
        if (deep) {
            if ((rc = flatten_all(c, totals + 5, htot + 8, &deep_rounds))) return rc;
            ++deep_rounds;
            e = hipMemsetAsync(totals + 4, 0, sizeof(unsigned long long), c.stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
        }
        // Shortcut: point the roots hooked since the last full flatten at
        // their roots, unless nothing survives or the pass's hooks far
        // outnumber the survivors (typically after the first pass, when nearly
        // every vertex was hooked): then the few survivors' finds walk the
        // extra links, and the final labelling flattens everything once.
        const bool jump = !deep && kept > 0 && fresh > 0 && hooks <= kLazyJump * kept;
        if (jump) {
            int k1 = c.kbeg();
            e = launch_sv_shortcut(c.parent, (const int32_t*)phook + (int64_t)jump_lo * cap, hooked_count + jump_lo,
                                   cap, nseg - jump_lo, c.stream);
            if (e != hipSuccess) return hip_fail(e, "sv_shortcut launch");
            c.kend(CC_K_SV_SHORTCUT, k1, 12.0 * fresh);
        }
        if (c.stats) {
            if (c.stats->sv_passes < 64) c.stats->active_edges[c.stats->sv_passes] = m_in;
            c.stats->sv_passes++;
            c.stats->hooks_total += hooks;
            c.stats->sv_atomics += natom;
            c.stats->sv_chase_reads += nchase;
            c.stats->giant_dropped += ndrop;
            if (pass == 0 && hubs_listed) c.stats->sv_hubs = (int32_t)std::min<uint32_t>((uint32_t)htot[11], kHubMax);
            // edges read (8 B) with two 4 B gathers (or bit probes) each, the
            // two parent gathers of the edges that passed the bitmap, 8 B per
            // atomic issued, 4 B per read of the walks up the forest, and the
            // survivors written (8 B); shortcut: read, gather, write per
            // hooked root
            const double rest = 8.0 * (double)(filt_edges - ndrop) + 8.0 * natom + 4.0 * nchase +
                                (write ? 8.0 * kept : 0.0);
            c.bytes += 16.0 * m_in + rest + (jump ? 12.0 * fresh : 0.0) + flat_bytes;
            c.kadd(rec_pass, rest);
        }
        ++pass;
        if (c.opt.check && (rc = check_parent(ws, c.stream, c.parent, c.n, pass))) return rc;
        if (kept == 0) break;
        in = out;
        in_soa = false;
        in_buf = out_buf;
        in_cnt = out_cnt;
        m_in = kept;
    }
    if ((rc = flatten_all(c, totals + 5, htot + 8, &deep_rounds))) return rc;
    if (c.stats) c.stats->sv_deep_rounds = deep_rounds;
    if (c.opt.check && c.stats) {
        // Section III-A: O(log n) iterations; far more marks a regression
        const int limit = 8 * (int)std::ceil(std::log2((double)c.n + 1.0)) + 64;
        c.stats->check_pass_limit = limit;
        if (pass > limit) c.stats->check_flags |= 2;
    }
    return CC_OK;
}

}  // namespace ccmi

using namespace ccmi;

// ------------------------------------------------------------------- C ABI
CC_API void cc_default_options(cc_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->route = CC_ROUTE_AUTO;
    opt->max_passes = 0;
    opt->tau = 0.05;
    opt->theta = 8.0;
}

CC_API int cc_version(void) { return CC_VERSION; }

CC_API const char* cc_last_error(void) { return g_err.c_str(); }

static void stats_reset(cc_stats* st) {
    memset(st, 0, sizeof *st);
    st->route = -1;
    st->bfs_seed = -1;
    st->bfs_label = -1;
    st->max_degree = -1;
    st->ks_statistic = NAN;
    st->ks_alpha = NAN;
}

CC_API int cc_label_ex(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream,
                       const cc_options* opt_in, cc_stats* stats) {
    g_err.clear();
    cc_options opt;
    if (opt_in) opt = *opt_in; else cc_default_options(&opt);
    if (opt.tau <= 0) opt.tau = 0.05;
    if (opt.theta < 1) opt.theta = 8.0;
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size (m=%lld, n=%d)", (long long)m, n);
    if (m > 0 && n == 0) return fail(CC_EINVAL, "edges given for an empty vertex set");
    if (m > 0 && (!u || !v)) return fail(CC_EINVAL, "NULL edge array");
    if (n > 0 && !labels) return fail(CC_EINVAL, "NULL labels");
    if (opt.route < CC_ROUTE_AUTO || opt.route > CC_ROUTE_SV_THETA) return fail(CC_EINVAL, "bad route %d", opt.route);
    if (opt.max_passes < 0) return fail(CC_EINVAL, "negative max_passes");
    if (m > (int64_t)2048 * (int64_t)INT32_MAX) return fail(CC_EINVAL, "too many edges");
    if (opt.workspace && opt.workspace_bytes <= 0) return fail(CC_EINVAL, "workspace given with no size");
    if (opt.scratch != CC_SCRATCH_POOL && opt.scratch != CC_SCRATCH_CACHED)
        return fail(CC_EINVAL, "bad scratch mode %d", opt.scratch);
    opt.check = check_enabled(opt);
    if (opt.max_passes == 0) {
        // CCMI_MAX_PASSES=k caps the SV passes of calls that set no cap (failure tests)
        const char* e = getenv("CCMI_MAX_PASSES");
        const int k = e ? atoi(e) : 0;
        if (k > 0) opt.max_passes = k;
    }
    if (stats) stats_reset(stats);
    if (n == 0) return CC_OK;

    // scratch: the caller's block, stream-ordered allocations from the
    // library's pool, or (the default) the library's cached per-device
    // buffers, serialised by their lock
    Workspace local;
    Workspace* ws = &local;
    std::unique_lock<std::mutex> lk;
    int rc;
    if (opt.workspace) {
        const bool sv_only = opt.route == CC_ROUTE_SV || opt.route == CC_ROUTE_SV_THETA;
        const size_t need = workspace_bound(m, n, sv_only, local.bound);
        if ((size_t)opt.workspace_bytes < need)
            return fail(CC_EINVAL, "workspace of %lld bytes is smaller than the %zu this call may need",
                        (long long)opt.workspace_bytes, need);
        hipError_t e = hipGetDevice(&local.device);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        local.mode = Workspace::kArena;
        local.arena = (char*)opt.workspace;
        local.arena_bytes = (size_t)opt.workspace_bytes;
    } else if (opt.scratch == CC_SCRATCH_POOL) {
        if ((rc = pool_workspace(&local, (hipStream_t)stream))) return rc;
    } else {
        if ((rc = acquire_workspace(&ws))) return rc;
        lk = std::unique_lock<std::mutex>(ws->mu);
    }

    Call c;
    c.ws = ws;
    c.stream = (hipStream_t)stream;
    c.n = n;
    c.m = m;
    c.u = u;
    c.v = v;
    c.parent = labels;
    c.stats = stats;
    c.opt = opt;
    Timer tm(stats != nullptr, c.stream);
    c.timer = &tm;
    int t0 = tm.mark();
    rc = run_label(c);
    int t1 = tm.mark();
    if (rc) return rc;
    if (opt.check) {
        if ((rc = check_result(*ws, c.stream, u, v, m, n, labels))) return rc;
        if (stats) {
            stats->check_flags |= 1;
            if (!stats->check_pass_limit)
                stats->check_pass_limit = 8 * (int)std::ceil(std::log2((double)n + 1.0)) + 64;
        }
    }
    if (stats) {
        stats->ms_total = tm.ms(t0, t1);
        stats->algorithmic_bytes = c.bytes;
        for (const auto& r : c.krecs) {
            if (r.cls < 0 || r.cls >= CC_K_CLASSES) continue;
            stats->kernel_ms[r.cls] += tm.ms(r.a, r.b);
            stats->kernel_launches[r.cls] += 1;
            stats->kernel_bytes[r.cls] += r.bytes;
        }
    }
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return CC_OK;
}

CC_API int cc_debug_fail_alloc(int64_t nth) {
    if (nth < 0) return fail(CC_EINVAL, "negative allocation count");
    g_fail_alloc.store(nth);
    return CC_OK;
}

CC_API int cc_label(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream) {
    return cc_label_ex(u, v, m, n, labels, stream, nullptr, nullptr);
}

CC_API int64_t cc_workspace_size(int64_t m, int32_t n, int32_t route) {
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size (m=%lld, n=%d)", (long long)m, n);
    if (route < CC_ROUTE_AUTO || route > CC_ROUTE_SV_THETA) return fail(CC_EINVAL, "bad route %d", route);
    return (int64_t)workspace_bound(m, n, route == CC_ROUTE_SV || route == CC_ROUTE_SV_THETA, nullptr);
}

CC_API int cc_release_workspace(void) {
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::lock_guard<std::mutex> guard(ws->mu);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    ws->release();
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto it = g_pools.find(ws->device);
    if (it != g_pools.end() && (e = hipMemPoolTrimTo(it->second, 0)) != hipSuccess)
        return hip_fail(e, "hipMemPoolTrimTo");
    return CC_OK;
}

// Everything the library holds, on every device it used: cached workspaces,
// memory pools, pinned staging, router copies.  No call may be running.
CC_API int cc_shutdown(void) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int rc = CC_OK;
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        for (auto& kv : g_ws) {
            if (hipSetDevice(kv.first) != hipSuccess) continue;
            std::lock_guard<std::mutex> wl(kv.second->mu);
            if ((e = hipDeviceSynchronize()) != hipSuccess && rc == CC_OK) rc = hip_fail(e, "hipDeviceSynchronize");
            kv.second->release();
        }
        for (auto& kv : g_pools) {
            if (hipSetDevice(kv.first) != hipSuccess) continue;
            if ((e = hipDeviceSynchronize()) != hipSuccess && rc == CC_OK) rc = hip_fail(e, "hipDeviceSynchronize");
            if ((e = hipMemPoolDestroy(kv.second)) != hipSuccess && rc == CC_OK) rc = hip_fail(e, "hipMemPoolDestroy");
        }
        g_pools.clear();
    }
    {
        std::lock_guard<std::mutex> g(g_side_mu);
        for (auto& kv : g_side) {
            if (hipSetDevice(kv.first) != hipSuccess) continue;
            if ((e = hipStreamDestroy(kv.second)) != hipSuccess && rc == CC_OK) rc = hip_fail(e, "hipStreamDestroy");
        }
        g_side.clear();
    }
    {
        std::lock_guard<std::mutex> g(g_stage_mu);
        for (void* p : g_stage_all) (void)hipHostFree(p);
        g_stage_all.clear();
        g_stage_free.clear();
    }
    router_release_all();
    (void)hipSetDevice(cur);
    return rc;
}
