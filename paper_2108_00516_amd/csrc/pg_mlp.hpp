// Learned correspondence weighting network (a 6-32-32-1 perceptron with ReLU
// hidden layers and a sigmoid output) shared by the association kernels, the
// pruning pass and the training kernels.  Parameter layout, 1313 values:
// W1 [32 x 6] row-major, b1 [32], W2 [32 x 32] row-major, b2 [32], W3 [32], b3.
#pragma once

#include <hip/hip_runtime.h>

namespace pg {

constexpr int kMlpIn = 6;
constexpr int kMlpHid = 32;
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpHid * kMlpIn;     // 192
constexpr int kMlpW2 = kMlpB1 + kMlpHid;              // 224
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;    // 1248
constexpr int kMlpW3 = kMlpB2 + kMlpHid;              // 1280
constexpr int kMlpB3 = kMlpW3 + kMlpHid;              // 1312
constexpr int kMlpParams = kMlpB3 + 1;                // 1313

// Logit of the network for input f.  P holds FP32 parameters; when every lane
// of a wave passes the same P, the parameter reads are uniform and go through
// the scalar cache into SGPRs.
__device__ __forceinline__ float mlp_logit(const float* __restrict__ P, const float (&f)[kMlpIn])
{
    float h1[kMlpHid];
#pragma unroll
    for (int o = 0; o < kMlpHid; ++o) {
        float s = P[kMlpB1 + o];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k)
            s = fmaf(P[kMlpW1 + kMlpIn * o + k], f[k], s);
        h1[o] = fmaxf(s, 0.0f);
    }
    float z = P[kMlpB3];
#pragma unroll 4
    for (int o = 0; o < kMlpHid; ++o) {
        float s = P[kMlpB2 + o];
#pragma unroll
        for (int k = 0; k < kMlpHid; ++k)
            s = fmaf(P[kMlpW2 + kMlpHid * o + k], h1[k], s);
        z = fmaf(P[kMlpW3 + o], fmaxf(s, 0.0f), z);
    }
    return z;
}

__device__ __forceinline__ float mlp_sigma(const float* __restrict__ P, const float (&f)[kMlpIn])
{
    return 1.0f / (1.0f + expf(-mlp_logit(P, f)));
}

}  // namespace pg
