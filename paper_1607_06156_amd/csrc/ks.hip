// Power-law fit of the degree distribution and its K-S statistic (Section
// III-B; Clauset, Shalizi & Newman, SIAM Review 2009, discrete case).
//
// The paper fits sequentially on each process (about a second for scale-free
// graphs) and names parallelising the fit as future work.  Here every
// candidate cutoff d_min is one workgroup:
//   * thread 0 solves the likelihood equation E_alpha[ln d | d >= d_min] =
//     mean(ln d_i) for alpha in (1, 10] by safeguarded Newton steps (the
//     derivative of E_alpha[ln d] is -Var_alpha[ln d]);
//   * all threads then evaluate the model CDF 1 - zeta(alpha, d+1)/zeta(alpha,
//     d_min) at every observed degree and just before the next one, and the
//     block reduces the largest gap to the empirical CDF (stopping early once
//     the candidate cannot be the best one).
// The Hurwitz zeta function and its first two s-derivatives come from the
// Euler-Maclaurin formula (direct terms up to argument 20, 7 Bernoulli
// corrections), in fp64.
#include <math.h>

#include "common.hpp"
#include "ks.hpp"

namespace ccmi {

constexpr int kKsBlock = 256;

struct Z3 {
    double z, d1, d2;
};

// Euler-Maclaurin for zeta(s, q): the terms (q + k)^-s are summed directly
// until the argument reaches a = q + N >= 20, and the tail from a is
// a^(1-s)/(s-1) + a^-s/2 + sum_j B_2j/(2j)! s(s+1)..(s+2j-2) a^(-s-2j+1),
// j = 1..7.  At a >= 20 the first omitted term is below 2e-14 of the sum for
// s <= 10.  The tail's powers of a come from one exp and multiplications by
// 1/a^2, so a large argument (a degree >= 20) costs one log and one exp.
__device__ __forceinline__ int direct_terms(double q) { return q < 20.0 ? (int)ceil(20.0 - q) : 0; }

// zeta(s, q) and its first two derivatives in s
__device__ Z3 hurwitz3(double s, double q) {
    const double C[7] = {1.0 / 6 / 2, -1.0 / 30 / 24, 1.0 / 42 / 720, -1.0 / 30 / 40320, 5.0 / 66 / 3628800,
                         -691.0 / 2730 / 479001600, 7.0 / 6 / 87178291200.0};
    double z = 0, d1 = 0, d2 = 0;
    const int N = direct_terms(q);
    for (int k = 0; k < N; ++k) {
        double L = log(q + k);
        double t = exp(-s * L);
        z += t;
        d1 -= L * t;
        d2 += L * L * t;
    }
    const double a = q + N, La = log(a);
    const double r = 1.0 / (s - 1.0);
    const double p0 = exp(-s * La);   // a^-s
    const double p1 = a * p0;         // a^(1-s)
    z += p1 * r;
    d1 += p1 * (-La * r - r * r);
    d2 += p1 * (La * La * r + 2.0 * La * r * r + 2.0 * r * r * r);
    z += 0.5 * p0;
    d1 -= 0.5 * La * p0;
    d2 += 0.5 * La * La * p0;
    const double ia2 = 1.0 / (a * a);
    double P = p0 / a;                // a^(-s-2j+1), j = 1
    double R = s, R1 = 1.0, R2 = 0.0;
    for (int j = 1; j <= 7; ++j) {
        const double c = C[j - 1];
        z += c * R * P;
        d1 += c * P * (R1 - La * R);
        d2 += c * P * (R2 - 2.0 * La * R1 + La * La * R);
        const double f1 = s + 2.0 * j - 1.0, f2 = s + 2.0 * j;
        const double nR2 = R2 * f1 * f2 + 2.0 * R1 * (f1 + f2) + 2.0 * R;
        const double nR1 = R1 * f1 * f2 + R * (f1 + f2);
        R = R * f1 * f2;
        R1 = nR1;
        R2 = nR2;
        P *= ia2;
    }
    return Z3{z, d1, d2};
}

__device__ double hurwitz(double s, double q) {
    const double C[7] = {1.0 / 6 / 2, -1.0 / 30 / 24, 1.0 / 42 / 720, -1.0 / 30 / 40320, 5.0 / 66 / 3628800,
                         -691.0 / 2730 / 479001600, 7.0 / 6 / 87178291200.0};
    double z = 0;
    const int N = direct_terms(q);
    for (int k = 0; k < N; ++k) z += exp(-s * log(q + k));
    const double a = q + N, La = log(a);
    const double p0 = exp(-s * La);
    z += a * p0 / (s - 1.0) + 0.5 * p0;
    const double ia2 = 1.0 / (a * a);
    double P = p0 / a, R = s;
    for (int j = 1; j <= 7; ++j) {
        z += C[j - 1] * R * P;
        R *= (s + 2.0 * j - 1.0) * (s + 2.0 * j);
        P *= ia2;
    }
    return z;
}

// E_alpha[ln d] - target and its derivative -Var_alpha[ln d]
__device__ void score(double a, double dmin, double target, double* f, double* fp) {
    Z3 t = hurwitz3(a, dmin);
    const double m1 = -t.d1 / t.z;        // E[ln d]
    const double m2 = t.d2 / t.z;         // E[(ln d)^2]
    *f = m1 - target;
    *fp = -(m2 - m1 * m1);
}

__device__ double solve_alpha(double dmin, double target) {
    double lo = kAlphaLo, hi = kAlphaHi, f, fp;
    score(hi, dmin, target, &f, &fp);
    if (f >= 0) return hi;                // the tail is lighter than any alpha <= 10
    double a = 1.0 + 1.0 / fmax(target - log(dmin - 0.5), 1e-3);
    if (!(a > lo && a < hi)) a = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        score(a, dmin, target, &f, &fp);
        if (f > 0) lo = a; else hi = a;
        double na = (fp < 0) ? a - f / fp : 0.5 * (lo + hi);
        if (!(na > lo && na < hi)) na = 0.5 * (lo + hi);
        if (fabs(na - a) <= 1e-15 * a || hi - lo <= 1e-15 * hi) {
            a = na;
            break;
        }
        a = na;
    }
    return a;
}

// One block per candidate c (tail starts at distinct value i0 = cand[c]).
// The statistic is a maximum over the observed degrees, and only the smallest
// one is wanted, so a candidate can stop as soon as its running maximum
// exceeds the smallest complete statistic found so far (*best, an fp64 bit
// pattern: non-negative doubles order like their bits).  Phase 0 evaluates
// every stride-th candidate in full to set *best; phase 1 evaluates the rest
// and drops those that exceed it (reported as +inf).  The minimising
// candidates, ties included, never exceed *best, so they are evaluated in
// full: the result is the same as without the cut.
__global__ __launch_bounds__(kKsBlock) void ks_fit_kernel(const double* __restrict__ vals,
                                                          const double* __restrict__ tail_n,
                                                          const double* __restrict__ tail_s, int32_t V,
                                                          const int32_t* __restrict__ cand, int32_t C,
                                                          int32_t stride, int32_t phase,
                                                          unsigned long long* __restrict__ best,
                                                          double* __restrict__ outD, double* __restrict__ outA) {
    __shared__ double sh_alpha, sh_z0;
    __shared__ double red[kKsBlock / 64];
    __shared__ int stop;
    const int c = phase == 0 ? blockIdx.x * stride : blockIdx.x;
    if (c >= C || (phase == 1 && c % stride == 0)) return;   // block-uniform
    const int i0 = cand[c];
    const double dmin = vals[i0];
    const double N = tail_n[i0];
    if (threadIdx.x == 0) {
        double a = solve_alpha(dmin, tail_s[i0] / N);
        sh_alpha = a;
        sh_z0 = hurwitz(a, dmin);
        stop = 0;
    }
    __syncthreads();
    const double a = sh_alpha, z0 = sh_z0;
    double dev = 0.0;
    for (int j0 = i0; j0 < V; j0 += kKsBlock) {
        // the bound is loaded first: its latency hides behind the evaluation
        const double bound = phase == 1 ? __longlong_as_double((long long)__hip_atomic_load(
                                              best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                                        : INFINITY;
        const int j = j0 + threadIdx.x;
        if (j < V) {
            // empirical CDF at vals[j]: share of the tail with degree <= vals[j]
            const double S = (N - (j + 1 < V ? tail_n[j + 1] : 0.0)) / N;
            const double Fat = 1.0 - hurwitz(a, vals[j] + 1.0) / z0;
            double d = fabs(S - Fat);
            if (j + 1 < V) {
                const double Fb = 1.0 - hurwitz(a, vals[j + 1]) / z0;
                d = fmax(d, fabs(S - Fb));
            }
            dev = fmax(dev, d);
        }
        if (phase == 1) {
            double w = dev;
            for (int o = 32; o > 0; o >>= 1) w = fmax(w, __shfl_xor(w, o));
            if (w > bound) __hip_atomic_store(&stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(&stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
                break;
        }
    }
    for (int o = 32; o > 0; o >>= 1) dev = fmax(dev, __shfl_xor(dev, o));
    if (lane_id() == 0) red[threadIdx.x >> 6] = dev;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int w = 0; w < kKsBlock / 64; ++w) b = fmax(b, red[w]);
        const bool cut = __hip_atomic_load(&stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
        outD[c] = cut ? INFINITY : b;
        outA[c] = a;
        if (!cut)
            __hip_atomic_fetch_min(best, (unsigned long long)__double_as_longlong(b), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// about this many candidates are evaluated in full first
constexpr int32_t kKsSample = 256;
// below this many CDF evaluations in all (sum over candidates of V - i0) one
// launch without the cut is faster than two (each pays the exponent solves)
constexpr int64_t kKsCutWork = (int64_t)8 << 20;

hipError_t launch_ks_fit(const double* vals, const double* tail_n, const double* tail_s, int32_t V,
                         const int32_t* cand, int32_t C, int64_t work, unsigned long long* best, double* outD,
                         double* outA, hipStream_t s) {
    if (C <= 0) return hipSuccess;
    const int32_t stride = (C > kKsSample && work > kKsCutWork) ? (C + kKsSample - 1) / kKsSample : 1;
    ks_fit_kernel<<<(C + stride - 1) / stride, kKsBlock, 0, s>>>(vals, tail_n, tail_s, V, cand, C, stride, 0, best,
                                                                 outD, outA);
    if (stride > 1)
        ks_fit_kernel<<<C, kKsBlock, 0, s>>>(vals, tail_n, tail_s, V, cand, C, stride, 1, best, outD, outA);
    return hipGetLastError();
}

}  // namespace ccmi
