// Host-side internals of libccmi shared by api.cpp and the route drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/cc.h"
#include "common.hpp"
#include "degree.hpp"

namespace ccmi {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// workspace slots (grow-only device buffers, one set per device)
enum WsSlot {
    WS_EDGES0 = 0,   // active edges, segment buffer A (int2)
    WS_EDGES1,       // active edges, segment buffer B (int2)
    WS_HOOKED,       // roots hooked in a pass (int32, segmented)
    WS_SEGCOUNT,     // per-segment counts (4 arrays of uint32)
    WS_TOTALS,       // small counters (u64)
    WS_DEG,          // degree (int32[n])
    WS_HIST,         // histograms: block partials + reduced
    WS_TAIL,         // degrees >= 4096
    WS_OFF,          // CSR offsets (int64[n+1]) and scan partials
    WS_CURSOR,       // CSR fill cursors (u64[n])
    WS_ADJ,          // CSR adjacency (int32[2m])
    WS_BITS,         // visited / frontier bitmaps
    WS_QUEUE,        // BFS queues
    WS_MLP,          // router parameters / features / logits
    WS_KS,           // power-law fit inputs and results
    WS_HISTOUT,      // reduced histograms, tail count, arg-max key
    WS_BATCH,        // batched-mode tables
    WS_GIANT,        // bitmap of the largest tree during a chunked first pass
    WS_R64_KEYS,     // 64-bit relabel: hash table keys, then the compact labels
    WS_R64_CID,      // 64-bit relabel: compact id of each slot
    WS_R64_EDGES,    // 64-bit relabel: edges as slots, then as compact ids
    WS_R64_FLAGS,    // 64-bit relabel: flags and the distinct-id count
    WS_R64_SCAN,     // 64-bit relabel: scan tile sums
    WS_NSLOTS
};

// Device scratch of a call, in one of three forms:
//  kCached : the library's per-device buffers, grown on demand with hipMalloc
//            and kept between calls (until cc_release_workspace); a caller
//            holds `mu` while it uses them;
//  kPool   : stream-ordered allocations from the library's per-device memory
//            pool on the call's stream, freed (stream-ordered) when the call
//            ends; the pool keeps the memory for later calls;
//  kArena  : a caller-provided block, cut into one region per slot, each
//            sized on its first use to the slot's bound for the call's (m, n)
//            (workspace_bound), so no request outgrows it.
// Small readbacks go through `host`: pinned staging of kHostBytes (kCached:
// the device's own; otherwise taken from a shared pool for the call), or a
// caller buffer marked host_external, large enough for the readbacks of the
// route it serves (cc_label_noalloc: 64 words for the SV route's counters).
struct Workspace {
    enum Mode { kCached = 0, kPool = 1, kArena = 2 };
    struct Buf {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    static constexpr size_t kHostBytes = 1 << 20;
    Mode mode = kCached;
    int device = 0;
    std::mutex mu;              // kCached only
    Buf bufs[WS_NSLOTS];
    void* host = nullptr;       // staging for small readbacks
    bool host_external = false; // host belongs to the caller
    bool host_leased = false;   // host came from the shared pinned pool
    // kPool
    hipStream_t stream = nullptr;
    hipMemPool_t pool = nullptr;
    // kArena
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    size_t bound[WS_NSLOTS] = {};
    ~Workspace();
    void release();
    int get(int slot, size_t bytes, void** out);
    int pinned(void** out);
    // end of a kPool / kArena call: free the pool allocations on `stream`
    // and return the pinned staging
    void finish();
};

// Upper bound of each slot's size for one cc_label_ex call on (m, n).
// sv_only: the routes without the degree pass (forced R1 / R2), whose scratch
// is the SV iteration's alone.  Returns the total, each region rounded up to
// 256 bytes, plus 256 for the alignment of the block itself.
size_t workspace_bound(int64_t m, int32_t n, bool sv_only, size_t* per_slot);

// a per-call workspace in kPool mode on the current device (stream-ordered)
int pool_workspace(Workspace* ws, hipStream_t s);

int acquire_workspace(Workspace** out);

// the device's second stream (created on first use, destroyed by cc_shutdown)
int side_stream(hipStream_t* out);

// true when a pending cc_debug_fail_alloc countdown makes this allocation fail
bool alloc_fault();

// debug checks (check.hip); counters live in the totals block from this word
constexpr int kCheckWords = 48;
int check_enabled(const cc_options& opt);
int check_parent(Workspace& ws, hipStream_t s, const int32_t* parent, int32_t n, int pass);
int check_labels(Workspace& ws, hipStream_t s, const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                 const int32_t* labels, int64_t bad[3], int64_t first[3]);
int check_result(Workspace& ws, hipStream_t s, const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                 const int32_t* labels);
// frees the router weights' device copies (router.cpp)
void router_release_all();

// An event that only times work: created without the system-scope fence a
// default event performs when it is recorded (a cache writeback and
// invalidation), so recording it between two kernels neither stalls the
// stream nor empties the L2 the next kernel reads from.
hipError_t create_timing_event(hipEvent_t* ev);

struct Timer {
    bool enabled;
    hipStream_t stream;
    std::vector<hipEvent_t> events;
    Timer(bool on, hipStream_t s);
    ~Timer();
    int mark();
    double ms(int a, int b);
};

// one cc_label_ex call
struct Call {
    Workspace* ws = nullptr;
    hipStream_t stream = nullptr;
    const int32_t* u = nullptr;
    const int32_t* v = nullptr;
    int64_t m = 0;
    int32_t n = 0;
    int32_t* parent = nullptr;  // = labels_out
    cc_stats* stats = nullptr;
    cc_options opt{};
    Timer* timer = nullptr;
    double bytes = 0.0;         // algorithmic bytes (cost model)
    bool range_checked = false;
    // step entry points may direct the degree pass's outputs into caller arrays
    int32_t* deg_out = nullptr;
    // degrees known before SV (heuristic route): hubs are the vertices of
    // degree >= hub_min, given a table in the first pass's filtered launches
    const int32_t* hub_deg = nullptr;
    int32_t hub_min = 0;
    int64_t* off_out = nullptr;
    int32_t* adj_out = nullptr;
    // per-kernel profiling (opt.profile with stats): event pairs per launch
    struct KRec {
        int cls, a, b;
        double bytes;
    };
    std::vector<KRec> krecs;
    bool profiling() const { return stats && opt.profile && timer; }
    int kbeg() { return profiling() ? timer->mark() : -1; }
    // returns the record index (or -1) so bytes can be filled in later
    int kend(int cls, int a, double kbytes) {
        if (!profiling()) return -1;
        int b = timer->mark();
        krecs.push_back(KRec{cls, a, b, kbytes});
        return (int)krecs.size() - 1;
    }
    // The end mark of record rec, or -1.  A group of kernels enqueued right
    // after another (nothing else in between) starts at that mark: one event
    // fewer on the stream per group.
    int kmark(int rec) const { return rec >= 0 ? krecs[rec].b : -1; }
    int kbeg_after(int mark) { return mark >= 0 ? mark : kbeg(); }
    void kbytes(int rec, double kbytes) {
        if (rec >= 0) krecs[rec].bytes = kbytes;
    }
    void kadd(int rec, double kbytes) {
        if (rec >= 0) krecs[rec].bytes += kbytes;
    }
};

struct SvInput {
    bool soa = true;
    const int32_t* u = nullptr;
    const int32_t* v = nullptr;
    int64_t m = 0;       // edges (dense count for soa, total active for seg)
    SegList seg{};       // when !soa: list in WS_EDGES0
};

// The first pass's first launch, enqueued ahead of the route decision.
struct SvSpec {
    bool launched = false;
    int rec = -1;          // its kernel record (profiling)
    int t0 = -1, t1 = -1;  // timer marks around it
};

int choose_nseg(int64_t m);
int pass0_chunks(int64_t m, int32_t n);
int sv_speculate(Call& c, const SvInput& in, SvSpec* spec);
// spec: resume after sv_speculate on the same list (its launch is not repeated)
int run_sv(Call& c, const SvInput& in, int policy, double theta, int max_passes, const SvSpec* spec = nullptr);
int run_label(Call& c);

// result of the degree pass (prediction step)
struct DegreeResult {
    BucketPlan plan{};
    BucketBufs bufs{};
    int32_t* deg = nullptr;
    int32_t* tail = nullptr;
    int64_t tail_cap = 0;
    unsigned long long* hist64_dev = nullptr;
    int64_t hist64[64] = {};
    std::vector<int64_t> histx;
    int64_t ntail = 0;
    int64_t max_degree = 0;
    int32_t argmax = -1;
    int64_t hub_min = 0;               // hub threshold from the power-law fit (0: none)
    bool csr_built = false;
    bool prefetch_tail = false;        // set by the caller: read the tail back with the histograms
    // set by the caller: enqueue this SV launch before waiting for the
    // histograms (sv_speculate on the caller's list)
    SvSpec* spec = nullptr;
    const int32_t* tail_host = nullptr;   // the first tail_host_n tail entries, in pinned host memory
    int64_t tail_host_n = 0;
    int64_t* off = nullptr;
    int32_t* adj = nullptr;
};

struct BfsResult {
    int levels = 0, bottom_up = 0;
    int64_t visited = 0, examined = 0;
    int64_t unvisited_entries = 0;   // adjacency entries in the rows of unvisited vertices
    bool abandoned = false;          // stopped at the level budget with the frontier not empty
};

int run_degree_pass(Call& c, bool want_csr, DegreeResult* r);
// max_levels > 0: stop after that many levels if the frontier is not empty yet
// (br->abandoned; the visited set is then incomplete)
int run_bfs(Call& c, const int64_t* off, const int32_t* adj, int64_t nadj, int32_t seed, int64_t seed_deg,
            int max_levels, uint32_t** vis_out, BfsResult* br);

}  // namespace ccmi
