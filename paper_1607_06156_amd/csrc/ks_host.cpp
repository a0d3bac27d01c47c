// Host side of the power-law fit: builds the degree distribution D from the
// device histograms, lists the candidate cutoffs and picks the best one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "degree.hpp"
#include "hubs.hpp"
#include "internal.hpp"
#include "ks.hpp"

namespace ccmi {

// ascending LSD radix sort, 11-bit digits, only as many passes as the largest
// value needs (a tail of ~13 000 degrees: about 0.1 ms, std::sort 0.7 ms)
static void radix_sort_u32(std::vector<uint32_t>& a) {
    uint32_t mx = 0;
    for (uint32_t x : a) mx = x > mx ? x : mx;
    std::vector<uint32_t> tmp(a.size());
    for (int shift = 0; shift < 32 && (mx >> shift) != 0; shift += 11) {
        uint32_t cnt[2048] = {0};
        for (uint32_t x : a) ++cnt[(x >> shift) & 2047u];
        uint32_t sum = 0;
        for (int i = 0; i < 2048; ++i) {
            const uint32_t c = cnt[i];
            cnt[i] = sum;
            sum += c;
        }
        for (uint32_t x : a) tmp[cnt[(x >> shift) & 2047u]++] = x;
        a.swap(tmp);
    }
}

// ln d of every exact-bin degree, computed once per process (the same values
// std::log gives on each call; a fit sums up to 4095 of them)
static const double* ln_exact() {
    static const std::vector<double> t = [] {
        std::vector<double> v(kExactBins, 0.0);
        for (int d = 1; d < kExactBins; ++d) v[d] = std::log((double)d);
        return v;
    }();
    return t.data();
}

int ks_fit(Workspace& ws, hipStream_t s, const int64_t* histx, const int32_t* tail, int64_t ntail, KsResult* out) {
    *out = KsResult{};
    // distinct positive degrees (ascending) and their vertex counts
    std::vector<double> vals;
    std::vector<double> cnts;
    vals.reserve((size_t)kExactBins + (size_t)std::max<int64_t>(ntail, 0));
    cnts.reserve(vals.capacity());
    for (int d = 1; d < kExactBins; ++d)
        if (histx[d] > 0) {
            vals.push_back((double)d);
            cnts.push_back((double)histx[d]);
        }
    if (ntail > 0) {
        // degrees >= 4096 (positive): sorted as unsigned
        std::vector<uint32_t> t((const uint32_t*)tail, (const uint32_t*)tail + ntail);
        radix_sort_u32(t);
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
    const double* lnx = ln_exact();
    double an = 0, as = 0;
    for (int32_t i = V - 1; i >= 0; --i) {
        an += cnts[i];
        as += cnts[i] * (vals[i] < kExactBins ? lnx[(int)vals[i]] : std::log(vals[i]));
        tn[i] = an;
        ts[i] = as;
    }
    for (int32_t i = 0; i < V; ++i)
        if (vals[i] >= (double)kHubMinDegree && tn[i] <= (double)kHubMax) {
            out->hub_min = (int64_t)vals[i];
            break;
        }
    std::vector<int32_t> cand;
    for (int32_t i = 0; i < V; ++i)
        if (tn[i] >= (double)kMinTail && V - i >= 2) cand.push_back(i);
    const int32_t C = (int32_t)cand.size();
    out->candidates = C;
    if (C == 0) return CC_OK;
    // device copies: vals, tail_n, tail_s (V doubles each), the running best
    // statistic (+inf bits), cand (C int32), then (8-byte aligned) the results
    // D, alpha (C doubles each).  The inputs go up in one copy and the results
    // come back in one, both through the pinned staging buffer when they fit.
    const size_t in_bytes = ((size_t)V * 3 + 1) * sizeof(double) + (size_t)C * sizeof(int32_t);
    const size_t res_off = (in_bytes + 7) & ~(size_t)7;
    const size_t res_bytes = (size_t)C * 2 * sizeof(double);
    void* dbuf;
    int rc = ws.get(WS_KS, res_off + res_bytes, &dbuf);
    if (rc) return rc;
    double* dv = (double*)dbuf;
    unsigned long long* dbest = (unsigned long long*)(dv + 3 * (size_t)V);
    int32_t* dc = (int32_t*)(dbest + 1);
    double* dD = (double*)((char*)dbuf + res_off);
    double* dA = dD + C;
    std::vector<char> pageable;
    char* h;
    if (res_off + res_bytes <= Workspace::kHostBytes) {
        void* hp;
        if ((rc = ws.pinned(&hp))) return rc;
        h = (char*)hp;
    } else {
        pageable.resize(res_off + res_bytes);
        h = pageable.data();
    }
    std::memcpy(h, vals.data(), V * sizeof(double));
    std::memcpy(h + V * sizeof(double), tn.data(), V * sizeof(double));
    std::memcpy(h + 2 * V * sizeof(double), ts.data(), V * sizeof(double));
    const double inf = INFINITY;
    std::memcpy(h + 3 * V * sizeof(double), &inf, sizeof(double));
    std::memcpy(h + (3 * V + 1) * sizeof(double), cand.data(), C * sizeof(int32_t));
    hipError_t e;
    if ((e = hipMemcpyAsync(dbuf, h, in_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(ks inputs)");
    int64_t work = 0;
    for (int32_t c = 0; c < C; ++c) work += V - cand[c];
    if ((e = launch_ks_fit(dv, dv + V, dv + 2 * (size_t)V, V, dc, C, work, dbest, dD, dA, s)) != hipSuccess)
        return hip_fail(e, "ks_fit launch");
    if ((e = hipMemcpyAsync(h + res_off, dD, res_bytes, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(ks results)");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const double* hD = (const double*)(h + res_off);
    const double* hA = hD + C;
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
