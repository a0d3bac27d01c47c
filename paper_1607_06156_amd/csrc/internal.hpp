// Host-side internals of libccmi shared by api.cpp and the route drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/cc.h"
#include "common.hpp"

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
    WS_BATCH,        // batched-mode tables
    WS_NSLOTS
};

struct Workspace {
    struct Buf {
        void* ptr = nullptr;
        size_t bytes = 0;
    };
    static constexpr size_t kHostBytes = 1 << 20;
    int device = 0;
    std::mutex mu;
    Buf bufs[WS_NSLOTS];
    void* host = nullptr;  // pinned staging for small readbacks
    ~Workspace();
    void release();
    int get(int slot, size_t bytes, void** out);
    int pinned(void** out);
};

int acquire_workspace(Workspace** out);

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
};

struct SvInput {
    bool soa = true;
    const int32_t* u = nullptr;
    const int32_t* v = nullptr;
    int64_t m = 0;       // edges (dense count for soa, total active for seg)
    SegList seg{};       // when !soa: list in WS_EDGES0
};

int run_sv(Call& c, const SvInput& in, int policy, double theta, int max_passes);
int run_label(Call& c);

}  // namespace ccmi
