// C ABI of the individual path steps (degree, histograms, power-law fit, CSR,
// BFS, label + filter), so each can be checked against the oracle on its own.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "bfs.hpp"
#include "degree.hpp"
#include "internal.hpp"
#include "ks.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

using namespace ccmi;

namespace {

struct Locked {
    Workspace* ws = nullptr;
    std::unique_lock<std::mutex> lk;
    int rc = CC_OK;
    Locked() {
        rc = acquire_workspace(&ws);
        if (rc == CC_OK) lk = std::unique_lock<std::mutex>(ws->mu);
    }
};

int finish(hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    return e == hipSuccess ? CC_OK : hip_fail(e, "hipStreamSynchronize");
}

}  // namespace

CC_API int cc_degree(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* deg, void* stream) {
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size");
    if (m > 0 && (!u || !v || n == 0)) return fail(CC_EINVAL, "bad edge arguments");
    if (n > 0 && !deg) return fail(CC_EINVAL, "NULL deg");
    if (n == 0) return CC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (m == 0) {
        hipError_t e = hipMemsetAsync(deg, 0, (size_t)n * sizeof(int32_t), s);
        return e == hipSuccess ? finish(s) : hip_fail(e, "hipMemsetAsync");
    }
    Locked L;
    if (L.rc) return L.rc;
    Call c;
    c.ws = L.ws;
    c.stream = s;
    c.u = u;
    c.v = v;
    c.m = m;
    c.n = n;
    c.deg_out = deg;
    Timer tm(false, s);
    c.timer = &tm;
    DegreeResult r;
    int rc = run_degree_pass(c, false, &r);
    return rc ? rc : finish(s);
}

CC_API int cc_degree_histograms(const int32_t* deg, int32_t n, int64_t* hist64, int64_t* histx, int32_t* tail,
                                int64_t tail_cap, int64_t* tail_count, int32_t* argmax, void* stream) {
    if (n < 0 || tail_cap < 0) return fail(CC_EINVAL, "negative size");
    if (!hist64 || !histx || (n > 0 && !deg) || (tail_cap > 0 && !tail)) return fail(CC_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    Locked L;
    if (L.rc) return L.rc;
    void* p;
    int rc = L.ws->get(WS_HISTOUT, 8 * sizeof(unsigned long long), &p);
    if (rc) return rc;
    unsigned long long* cnt = (unsigned long long*)p;   // [0] tail count, [1] arg-max key
    hipError_t e = hipMemsetAsync(hist64, 0, 64 * sizeof(int64_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(histx, 0, kExactBins * sizeof(int64_t), s);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), s);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    if (n > 0) {
        e = launch_degree_hist(deg, n, (unsigned long long*)hist64, (unsigned long long*)histx, tail, tail_cap,
                               cnt, cnt + 1, s);
        if (e != hipSuccess) return hip_fail(e, "degree_hist launch");
    }
    unsigned long long* host;
    if ((rc = L.ws->pinned((void**)&host))) return rc;
    e = hipMemcpyAsync(host, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "histogram readback");
    if (tail_count) *tail_count = (int64_t)host[0];
    if (argmax) {
        const unsigned long long key = host[1];
        *argmax = (n > 0) ? (int32_t)(~(uint32_t)(key & 0xffffffffull)) : -1;
        if (n > 0 && key == 0) *argmax = -1;
    }
    return CC_OK;
}

CC_API int cc_powerlaw_ks(const int64_t* histx, const int32_t* tail, int64_t ntail, double* out) {
    if (!histx || !out || ntail < 0 || (ntail > 0 && !tail)) return fail(CC_EINVAL, "bad arguments");
    for (int64_t i = 0; i < ntail; ++i)
        if (tail[i] < kExactBins) return fail(CC_EINVAL, "tail[%lld] = %d is below %d", (long long)i, tail[i], kExactBins);
    Locked L;
    if (L.rc) return L.rc;
    KsResult k;
    int rc = ks_fit(*L.ws, nullptr, histx, tail, ntail, &k);
    if (rc) return rc;
    out[0] = k.ks;
    out[1] = k.alpha;
    out[2] = (double)k.dmin;
    out[3] = (double)k.ntail;
    out[4] = (double)k.candidates;
    return CC_OK;
}

CC_API int cc_csr(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* deg, int64_t* off,
                  int32_t* adj, void* stream) {
    if (m < 0 || n < 0) return fail(CC_EINVAL, "negative size");
    if (m > 0 && (!u || !v || n == 0 || !adj)) return fail(CC_EINVAL, "bad edge arguments");
    if (!off) return fail(CC_EINVAL, "NULL off");
    hipStream_t s = (hipStream_t)stream;
    if (m == 0) {
        hipError_t e = hipMemsetAsync(off, 0, (size_t)(n + 1) * sizeof(int64_t), s);
        if (e == hipSuccess && deg && n) e = hipMemsetAsync(deg, 0, (size_t)n * sizeof(int32_t), s);
        return e == hipSuccess ? finish(s) : hip_fail(e, "hipMemsetAsync");
    }
    Locked L;
    if (L.rc) return L.rc;
    Call c;
    c.ws = L.ws;
    c.stream = s;
    c.u = u;
    c.v = v;
    c.m = m;
    c.n = n;
    c.deg_out = deg;
    c.off_out = off;
    c.adj_out = adj;
    Timer tm(false, s);
    c.timer = &tm;
    DegreeResult r;
    int rc = run_degree_pass(c, true, &r);
    return rc ? rc : finish(s);
}

CC_API int cc_bfs(const int64_t* off, const int32_t* adj, int32_t n, int64_t nadj, int32_t seed, uint32_t* visited,
                  int32_t* levels, int32_t* bottom_up, void* stream) {
    if (n <= 0 || nadj < 0 || !off || !visited || (nadj > 0 && !adj)) return fail(CC_EINVAL, "bad arguments");
    if (seed < 0 || seed >= n) return fail(CC_EINVAL, "seed %d outside [0, %d)", seed, n);
    hipStream_t s = (hipStream_t)stream;
    Locked L;
    if (L.rc) return L.rc;
    void* p;
    int rc = L.ws->get(WS_HISTOUT, 8 * sizeof(unsigned long long), &p);
    if (rc) return rc;
    unsigned long long* bad = (unsigned long long*)p;
    int64_t* hoff;
    if ((rc = L.ws->pinned((void**)&hoff))) return rc;
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), s);
    if (e == hipSuccess) e = launch_csr_check(off, n, adj, nadj, bad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hoff, bad, sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hoff + 1, off + seed, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "csr check");
    if (hoff[0]) return fail(CC_EINVAL, "CSR is malformed (%lld violations)", (long long)hoff[0]);
    const int64_t sdeg = hoff[2] - hoff[1];
    Call c;
    c.ws = L.ws;
    c.stream = s;
    c.n = n;
    c.m = nadj / 2;
    Timer tm(false, s);
    c.timer = &tm;
    uint32_t* vis = nullptr;
    BfsResult br;
    rc = run_bfs(c, off, adj, nadj, seed, sdeg, 0, &vis, &br);
    if (rc) return rc;
    e = hipMemcpyAsync(visited, vis, (size_t)(((int64_t)n + 31) >> 5) * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(visited)");
    if (levels) *levels = br.levels;
    if (bottom_up) *bottom_up = br.bottom_up;
    return finish(s);
}

CC_API int cc_bfs_filter(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const uint32_t* visited,
                         int32_t* labels, int32_t* fu, int32_t* fv, int64_t* m_kept, int32_t* label, void* stream) {
    if (m < 0 || n <= 0 || !visited || !labels) return fail(CC_EINVAL, "bad arguments");
    if (m > 0 && (!u || !v || !fu || !fv)) return fail(CC_EINVAL, "NULL edge array");
    hipStream_t s = (hipStream_t)stream;
    Locked L;
    if (L.rc) return L.rc;
    const int nseg = choose_nseg(m);
    const int64_t cap = m > 0 ? (m + nseg - 1) / nseg : 1;
    void *pe, *pc, *pt;
    int rc;
    if ((rc = L.ws->get(WS_EDGES0, (size_t)nseg * cap * sizeof(int2), &pe))) return rc;
    if ((rc = L.ws->get(WS_SEGCOUNT, (size_t)nseg * 4 * sizeof(uint32_t) + (size_t)(nseg + 2) * sizeof(int64_t),
                        &pc)))
        return rc;
    if ((rc = L.ws->get(WS_HISTOUT, 8 * sizeof(unsigned long long), &pt))) return rc;
    uint32_t* cnt = (uint32_t*)pc;
    int64_t* prefix = (int64_t*)((char*)pc + (size_t)nseg * 4 * sizeof(uint32_t));
    unsigned long long* tot = (unsigned long long*)pt;
    int32_t* dlabel = (int32_t*)(tot + 2);
    SegList out{(int2*)pe, cap, nseg, cnt};
    hipError_t e = hipMemsetAsync(tot, 0, 4 * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = hipMemsetAsync(dlabel, 0x7f, sizeof(int32_t), s);
    if (e == hipSuccess) e = launch_bfs_label(visited, n, dlabel, labels, s);
    if (e == hipSuccess && m > 0) e = launch_filter(u, v, m, n, visited, out, tot, tot + 1, s);
    if (e == hipSuccess && m > 0) e = launch_seg_to_soa(out, prefix, prefix + nseg + 1, fu, fv, s);
    if (e != hipSuccess) return hip_fail(e, "bfs_filter launch");
    unsigned long long* host;
    if ((rc = L.ws->pinned((void**)&host))) return rc;
    e = hipMemcpyAsync(host, tot, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "bfs_filter readback");
    if (host[1]) return fail(CC_ERANGE, "%llu edges have an endpoint outside [0, n)", host[1]);
    const int32_t lab = *(int32_t*)(host + 2);
    if (m_kept) *m_kept = (int64_t)host[0];
    if (label) *label = (lab >= n || lab < 0) ? -1 : lab;
    return CC_OK;
}
