// Power-law fit interface (ks.hip + ks_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ccmi {

constexpr double kAlphaLo = 1.0 + 1e-9;
constexpr double kAlphaHi = 10.0;
constexpr int64_t kMinTail = 50;   // vertices at or above a candidate cutoff

// outD[c], outA[c]: statistic and exponent of candidate c; a candidate that
// cannot have the smallest statistic may report +inf.  *best must hold the bits
// of +inf on entry; it ends as the bits of the smallest statistic.  work: the
// number of CDF evaluations, sum over candidates of V - cand[c].
hipError_t launch_ks_fit(const double* vals, const double* tail_n, const double* tail_s, int32_t V,
                         const int32_t* cand, int32_t C, int64_t work, unsigned long long* best, double* outD,
                         double* outA, hipStream_t s);

struct KsResult {
    double ks = INFINITY;
    double alpha = NAN;
    int64_t dmin = 0;
    int64_t ntail = 0;
    int64_t candidates = 0;
    // the smallest distinct degree d >= kHubMinDegree with at most kHubMax
    // vertices of degree >= d (0: none), the hub threshold of the first SV pass
    int64_t hub_min = 0;
};

struct Workspace;
// histx: host int64[4096]; tail: host int32[ntail] (degrees >= 4096, any order)
int ks_fit(Workspace& ws, hipStream_t s, const int64_t* histx, const int32_t* tail, int64_t ntail, KsResult* out);

}  // namespace ccmi
