// Router weights, the learned route decision, and the C ABI of the MLP kernels.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "router.hpp"

#define CC_API extern "C" __attribute__((visibility("default")))

namespace ccmi {

static std::mutex g_router_mu;
static std::vector<float> g_router;                  // host copy; empty = not loaded
static std::unordered_map<int, float*> g_router_dev;  // per-device copies
static uint64_t g_router_gen = 0;
static std::unordered_map<int, uint64_t> g_router_dev_gen;

bool router_loaded() {
    std::lock_guard<std::mutex> g(g_router_mu);
    return !g_router.empty();
}

static int router_device_params(float** out, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_router_mu);
    if (g_router.empty()) return fail(CC_ENOROUTER, "no router weights loaded");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    float*& p = g_router_dev[dev];
    if (!p) {
        e = alloc_fault() ? hipErrorOutOfMemory : hipMalloc(&p, kNParams * sizeof(float));
        if (e != hipSuccess) {
            p = nullptr;
            return hip_fail(e, "hipMalloc(router)");
        }
        g_router_dev_gen[dev] = ~0ull;
    }
    if (g_router_dev_gen[dev] != g_router_gen) {
        e = hipMemcpyAsync(p, g_router.data(), kNParams * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(router)");
        g_router_dev_gen[dev] = g_router_gen;
    }
    *out = p;
    return CC_OK;
}

// frees the per-device copies of the weights (the host copy stays loaded)
void router_release_all() {
    std::lock_guard<std::mutex> g(g_router_mu);
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto& kv : g_router_dev) {
        if (kv.second && hipSetDevice(kv.first) == hipSuccess) (void)hipFree(kv.second);
        kv.second = nullptr;
        g_router_dev_gen[kv.first] = ~0ull;
    }
    if (have_cur) (void)hipSetDevice(cur);
}

int decide_router(Call& c, DegreeResult& r, int* route) {
    float* P;
    int rc = router_device_params(&P, c.stream);
    if (rc) return rc;
    void* buf;
    if ((rc = c.ws->get(WS_MLP, (kF + 4) * sizeof(float), &buf))) return rc;
    float* x = (float*)buf;
    float* z = x + kF;
    hipError_t e = launch_router_features(r.hist64_dev, c.n, c.m, x, c.stream);
    if (e == hipSuccess) e = launch_mlp_forward(P, x, 1, z, c.stream);
    if (e != hipSuccess) return hip_fail(e, "router launch");
    float* host;
    if ((rc = c.ws->pinned((void**)&host))) return rc;
    e = hipMemcpyAsync(host, z, kO * sizeof(float), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return hip_fail(e, "router readback");
    int best = 0;
    for (int k = 1; k < kO; ++k)
        if (host[k] > host[best]) best = k;
    if (c.stats)
        for (int k = 0; k < kO; ++k) c.stats->router_logits[k] = host[k];
    *route = best;   // class k is route id k (CC_R0_BFS_SV, CC_R1_SV, CC_R2_SV_THETA)
    return CC_OK;
}

}  // namespace ccmi

using namespace ccmi;

CC_API int cc_router_set(const float* host_params) {
    std::lock_guard<std::mutex> g(g_router_mu);
    if (!host_params) {
        g_router.clear();
    } else {
        g_router.assign(host_params, host_params + kNParams);
    }
    ++g_router_gen;
    return CC_OK;
}

// Text weights: lines starting with '#' are comments; every other token,
// separated by blanks, is one number, and all kNParams of them must be
// finite.  Lines may be of any length.
CC_API int cc_router_load(const char* path) {
    if (!path) return fail(CC_EINVAL, "NULL path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(CC_EINVAL, "cannot open %s", path);
    std::vector<float> w;
    std::string tok;
    bool comment = false, line_start = true;
    int rc = CC_OK;
    auto flush = [&]() {
        if (tok.empty() || rc) return;
        char* end = nullptr;
        errno = 0;
        const float x = strtof(tok.c_str(), &end);
        if (end == tok.c_str() || *end != '\0' || !std::isfinite(x) || errno == ERANGE)
            rc = fail(CC_EINVAL, "%s: '%.40s' after %zu numbers is not a finite number", path, tok.c_str(),
                      w.size());
        else
            w.push_back(x);
        tok.clear();
    };
    for (int ch; (ch = fgetc(f)) != EOF && !rc;) {
        if (line_start && ch == '#') comment = true;
        line_start = ch == '\n';
        if (ch == '\n') {
            flush();
            comment = false;
        } else if (comment) {
            continue;
        } else if (ch == ' ' || ch == '\t' || ch == '\r') {
            flush();
        } else {
            tok.push_back((char)ch);
        }
    }
    flush();
    fclose(f);
    if (rc) return rc;
    if ((int)w.size() != kNParams)
        return fail(CC_EINVAL, "%s holds %zu numbers, expected %d", path, w.size(), kNParams);
    return cc_router_set(w.data());
}

CC_API int cc_router_loaded(void) { return router_loaded() ? 1 : 0; }

CC_API int cc_mlp_forward(const float* params, const float* x, int32_t batch, float* logits, void* stream) {
    if (batch < 0) return fail(CC_EINVAL, "negative batch");
    if (batch == 0) return CC_OK;
    if (!params || !x || !logits) return fail(CC_EINVAL, "NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_mlp_forward(params, x, batch, logits, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "mlp_forward");
    return CC_OK;
}

CC_API int cc_mlp_sgd_step(float* params, const float* x, const int32_t* y, int32_t batch, float lr, float* grads,
                           float* loss, void* stream) {
    if (batch <= 0) return fail(CC_EINVAL, "batch must be positive");
    if (!params || !x || !y) return fail(CC_EINVAL, "NULL pointer");
    Workspace* ws;
    int rc = acquire_workspace(&ws);
    if (rc) return rc;
    std::lock_guard<std::mutex> guard(ws->mu);
    hipStream_t s = (hipStream_t)stream;
    const size_t act = (size_t)batch * (4 * kH + kO);
    void* buf;
    if ((rc = ws->get(WS_MLP, (act + batch + kNParams + 4) * sizeof(float), &buf))) return rc;
    float* pact = (float*)buf;
    float* loss_b = pact + act;
    float* g = grads ? grads : loss_b + batch;
    float* dloss = (grads ? loss_b + batch : g + kNParams);
    hipError_t e = launch_mlp_grad(params, x, y, batch, g, loss_b, pact, s);
    if (e == hipSuccess) e = launch_mlp_update(params, g, lr, loss_b, batch, dloss, s);
    if (e != hipSuccess) return hip_fail(e, "mlp_sgd_step");
    float* host;
    if ((rc = ws->pinned((void**)&host))) return rc;
    e = hipMemcpyAsync(host, dloss, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "mlp loss readback");
    if (loss) *loss = host[0];
    return CC_OK;
}
