// Router network kernels: FP32 MLP 66 -> 64 -> 64 -> 3 with ReLU, softmax
// cross-entropy and plain SGD.  Everything is small (8643 parameters), so the
// kernels use ordinary FP32 FMA: one wave per sample for the forward and
// backward sweeps, one thread per parameter for the batch reduction of the
// gradient (deterministic order), no matrix cores.
#include <math.h>

#include "common.hpp"
#include "router.hpp"

namespace ccmi {

// per-sample activation record in `act`: a1[64] h1[64] a2[64] h2[64] dz[3]
constexpr int kAct = 4 * kH + kO;

__global__ void router_features_kernel(const unsigned long long* __restrict__ hist64, int64_t n, int64_t m,
                                       float* __restrict__ x) {
    int t = threadIdx.x;
    const double nn = n > 0 ? (double)n : 1.0;
    if (t < 64) x[t] = (float)((double)hist64[t] / nn);
    if (t == 64) x[64] = (float)log2(nn);
    if (t == 65) x[65] = (float)log2(m > 0 ? (double)m : 1.0);
}

// one 64-thread block per sample; returns h2 in LDS and optionally stores the record
__device__ void mlp_forward_sample(const float* __restrict__ P, const float* __restrict__ xin, float* xs, float* h1s,
                                   float* h2s, float* z, float* rec) {
    const int t = threadIdx.x;
    xs[t] = xin[t];
    if (t < kF - 64) xs[64 + t] = xin[64 + t];
    __syncthreads();
    float a = P[kOffB1 + t];
    const float* w1 = P + kOffW1 + t * kF;
    for (int i = 0; i < kF; ++i) a = fmaf(w1[i], xs[i], a);
    float h = a > 0.f ? a : 0.f;
    h1s[t] = h;
    if (rec) { rec[t] = a; rec[kH + t] = h; }
    __syncthreads();
    float a2 = P[kOffB2 + t];
    const float* w2 = P + kOffW2 + t * kH;
    for (int i = 0; i < kH; ++i) a2 = fmaf(w2[i], h1s[i], a2);
    float g = a2 > 0.f ? a2 : 0.f;
    h2s[t] = g;
    if (rec) { rec[2 * kH + t] = a2; rec[3 * kH + t] = g; }
    __syncthreads();
    if (t < kO) {
        float o = P[kOffB3 + t];
        const float* w3 = P + kOffW3 + t * kH;
        for (int i = 0; i < kH; ++i) o = fmaf(w3[i], h2s[i], o);
        z[t] = o;
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ x,
                                                         int32_t B, float* __restrict__ logits) {
    __shared__ float xs[kF], h1s[kH], h2s[kH], z[kO];
    const int b = blockIdx.x;
    mlp_forward_sample(P, x + (int64_t)b * kF, xs, h1s, h2s, z, nullptr);
    if (threadIdx.x < kO) logits[(int64_t)b * kO + threadIdx.x] = z[threadIdx.x];
}

// forward + per-sample backward: stores a1,h1,a2,h2 and the per-sample deltas
// (dz, da2, da1 overwrite dz-slot and a2/a1 slots after use)
__global__ __launch_bounds__(64) void mlp_backward_sample_kernel(const float* __restrict__ P,
                                                                 const float* __restrict__ x,
                                                                 const int32_t* __restrict__ y, int32_t B,
                                                                 float* __restrict__ act, float* __restrict__ loss_b) {
    __shared__ float xs[kF], h1s[kH], h2s[kH], z[kO], dz[kO], da2[kH];
    const int b = blockIdx.x, t = threadIdx.x;
    float* rec = act + (int64_t)b * kAct;
    mlp_forward_sample(P, x + (int64_t)b * kF, xs, h1s, h2s, z, rec);
    if (t == 0) {
        const float zm = fmaxf(z[0], fmaxf(z[1], z[2]));
        const float e0 = expf(z[0] - zm), e1 = expf(z[1] - zm), e2 = expf(z[2] - zm);
        const float s = e0 + e1 + e2;
        const int yy = y[b];
        const float inv = 1.f / (float)B;
        float p[3] = {e0 / s, e1 / s, e2 / s};
        loss_b[b] = -logf(p[yy]);
        for (int k = 0; k < kO; ++k) {
            float d = (p[k] - (k == yy ? 1.f : 0.f)) * inv;
            dz[k] = d;
            rec[4 * kH + k] = d;
        }
    }
    __syncthreads();
    // da2[j] = (sum_k dz[k] W3[k][j]) * (a2[j] > 0)
    float s2 = 0.f;
    for (int k = 0; k < kO; ++k) s2 = fmaf(dz[k], P[kOffW3 + k * kH + t], s2);
    const float a2v = rec[2 * kH + t];
    const float d2 = a2v > 0.f ? s2 : 0.f;
    da2[t] = d2;
    __syncthreads();
    // da1[i] = (sum_j da2[j] W2[j][i]) * (a1[i] > 0)
    float s1 = 0.f;
    for (int j = 0; j < kH; ++j) s1 = fmaf(da2[j], P[kOffW2 + j * kH + t], s1);
    const float a1v = rec[t];
    const float d1 = a1v > 0.f ? s1 : 0.f;
    __syncthreads();
    rec[t] = d1;            // a1 slot <- da1
    rec[2 * kH + t] = d2;   // a2 slot <- da2
}

// one thread per parameter: batch sums in a fixed order
__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float* __restrict__ x,
                                                              const float* __restrict__ act, int32_t B,
                                                              float* __restrict__ g) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParams) return;
    float s = 0.f;
    if (p < kOffB1) {
        const int i = p / kF, f = p % kF;        // gW1[i][f] = sum_b da1[b][i] x[b][f]
        for (int b = 0; b < B; ++b) s = fmaf(act[(int64_t)b * kAct + i], x[(int64_t)b * kF + f], s);
    } else if (p < kOffW2) {
        const int i = p - kOffB1;                // gb1[i] = sum_b da1[b][i]
        for (int b = 0; b < B; ++b) s += act[(int64_t)b * kAct + i];
    } else if (p < kOffB2) {
        const int q = p - kOffW2, j = q / kH, i = q % kH;   // gW2[j][i] = sum_b da2[b][j] h1[b][i]
        for (int b = 0; b < B; ++b)
            s = fmaf(act[(int64_t)b * kAct + 2 * kH + j], act[(int64_t)b * kAct + kH + i], s);
    } else if (p < kOffW3) {
        const int j = p - kOffB2;
        for (int b = 0; b < B; ++b) s += act[(int64_t)b * kAct + 2 * kH + j];
    } else if (p < kOffB3) {
        const int q = p - kOffW3, k = q / kH, j = q % kH;   // gW3[k][j] = sum_b dz[b][k] h2[b][j]
        for (int b = 0; b < B; ++b)
            s = fmaf(act[(int64_t)b * kAct + 4 * kH + k], act[(int64_t)b * kAct + 3 * kH + j], s);
    } else {
        const int k = p - kOffB3;
        for (int b = 0; b < B; ++b) s += act[(int64_t)b * kAct + 4 * kH + k];
    }
    g[p] = s;
}

__global__ __launch_bounds__(256) void mlp_update_kernel(float* __restrict__ P, const float* __restrict__ g, float lr,
                                                         const float* __restrict__ loss_b, int32_t B,
                                                         float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) P[p] -= lr * g[p];
    if (p == 0) {
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += loss_b[b];
        *loss = s / (float)B;
    }
}

hipError_t launch_router_features(const unsigned long long* hist64, int64_t n, int64_t m, float* x, hipStream_t s) {
    router_features_kernel<<<1, 128, 0, s>>>(hist64, n, m, x);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* x, int32_t B, float* logits, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    mlp_forward_kernel<<<B, 64, 0, s>>>(params, x, B, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* x, const int32_t* y, int32_t B, float* grads,
                           float* loss_b, float* act, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    mlp_backward_sample_kernel<<<B, 64, 0, s>>>(params, x, y, B, act, loss_b);
    mlp_grad_reduce_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(x, act, B, grads);
    return hipGetLastError();
}

hipError_t launch_mlp_update(float* params, const float* grads, float lr, const float* loss_b, int32_t B,
                             float* loss, hipStream_t s) {
    mlp_update_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(params, grads, lr, loss_b, B, loss);
    return hipGetLastError();
}

}  // namespace ccmi
