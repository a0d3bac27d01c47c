// Host side of the power-law fit: builds the degree distribution D from the
// device histograms, lists the candidate cutoffs and picks the best one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "degree.hpp"
#include "internal.hpp"
#include "ks.hpp"

namespace ccmi {

int ks_fit(Workspace& ws, hipStream_t s, const int64_t* histx, const int32_t* tail, int64_t ntail, KsResult* out) {
    *out = KsResult{};
    // distinct positive degrees (ascending) and their vertex counts
    std::vector<double> vals;
    std::vector<double> cnts;
    for (int d = 1; d < kExactBins; ++d)
        if (histx[d] > 0) {
            vals.push_back((double)d);
            cnts.push_back((double)histx[d]);
        }
    if (ntail > 0) {
        std::vector<int32_t> t(tail, tail + ntail);
        std::sort(t.begin(), t.end());
        for (size_t i = 0; i < t.size();) {
            size_t j = i;
            while (j < t.size() && t[j] == t[i]) ++j;
            vals.push_back((double)t[i]);
            cnts.push_back((double)(j - i));
            i = j;
        }
    }
    const int32_t V = (int32_t)vals.size();
    if (V < 2) return CC_OK;
    // suffix sums: vertices and sum of ln d at or above each distinct value
    std::vector<double> tn(V), ts(V);
    double an = 0, as = 0;
    for (int32_t i = V - 1; i >= 0; --i) {
        an += cnts[i];
        as += cnts[i] * std::log(vals[i]);
        tn[i] = an;
        ts[i] = as;
    }
    std::vector<int32_t> cand;
    for (int32_t i = 0; i < V; ++i)
        if (tn[i] >= (double)kMinTail && V - i >= 2) cand.push_back(i);
    const int32_t C = (int32_t)cand.size();
    out->candidates = C;
    if (C == 0) return CC_OK;
    // device copies: vals, tail_n, tail_s (V doubles each), cand, D, alpha
    size_t bytes = (size_t)V * 3 * sizeof(double) + (size_t)C * (sizeof(int32_t) + 2 * sizeof(double)) + 64;
    void* dbuf;
    int rc = ws.get(WS_KS, bytes, &dbuf);
    if (rc) return rc;
    double* dv = (double*)dbuf;
    double* dn = dv + V;
    double* dsum = dn + V;
    double* dD = dsum + V;
    double* dA = dD + C;
    int32_t* dc = (int32_t*)(dA + C);
    hipError_t e;
    if ((e = hipMemcpyAsync(dv, vals.data(), V * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dn, tn.data(), V * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dsum, ts.data(), V * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dc, cand.data(), C * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(ks inputs)");
    if ((e = launch_ks_fit(dv, dn, dsum, V, dc, C, dD, dA, s)) != hipSuccess) return hip_fail(e, "ks_fit launch");
    std::vector<double> hD(C), hA(C);
    if ((e = hipMemcpyAsync(hD.data(), dD, C * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(hA.data(), dA, C * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(ks results)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    int best = -1;
    for (int c = 0; c < C; ++c)
        if (best < 0 || hD[c] < hD[best]) best = c;
    out->ks = hD[best];
    out->alpha = hA[best];
    out->dmin = (int64_t)vals[cand[best]];
    out->ntail = (int64_t)tn[cand[best]];
    return CC_OK;
}

}  // namespace ccmi
