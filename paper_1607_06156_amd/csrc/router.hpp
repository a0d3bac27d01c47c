// Learned route selection: FP32 MLP 66 -> 64 -> 64 -> 3 (mlp.hip, router.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccmi {

constexpr int kF = 66, kH = 64, kO = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kF;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kO * kH;
constexpr int kNParams = kOffB3 + kO;

// features[66] from the device log-degree histogram (int64[64]) and n, m
hipError_t launch_router_features(const unsigned long long* hist64, int64_t n, int64_t m, float* x, hipStream_t s);
// logits[B][3] = MLP(x[B][66])
hipError_t launch_mlp_forward(const float* params, const float* x, int32_t B, float* logits, hipStream_t s);
// gradient of the mean cross-entropy into grads[kNParams]; per-sample loss into loss_b[B]
// (scratch: act = B * (2*kH + 2*kH + kO) floats)
hipError_t launch_mlp_grad(const float* params, const float* x, const int32_t* y, int32_t B, float* grads,
                           float* loss_b, float* act, hipStream_t s);
// params -= lr * grads; *loss = mean(loss_b)
hipError_t launch_mlp_update(float* params, const float* grads, float lr, const float* loss_b, int32_t B,
                             float* loss, hipStream_t s);

struct Call;
struct DegreeResult;
bool router_loaded();
int decide_router(Call& c, DegreeResult& r, int* route);

}  // namespace ccmi
