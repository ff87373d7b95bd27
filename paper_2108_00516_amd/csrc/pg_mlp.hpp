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

// ---------------------------------------------------------------------------
// The network on the matrix cores, one wave = 64 samples (one per lane), as
// the dense term evaluates it, "in FP16": every layer's input (the features
// and both hidden layers' activations) is a binary16 value, rounded to
// nearest with ties to even, the parameters are binary16, and each layer's
// products are summed in FP32 (the two hidden layers on
// v_mfma_f32_32x32x16_f16, the 32-term output layer on the vector units).
// Both hidden layers are computed transposed (hidden units as rows, samples
// as columns), so the first layer's output registers are already the second
// layer's B operand: a 32x32x16 product leaves row 8j + 4(lane/32) + i,
// column lane%32 in c[4j + i], and the two K steps of the second layer take
// c[0..7] and c[8..15] when the second layer's A operand (W2) has its hidden
// index permuted to match (hid = 8(2s + t/4) + 4(lane/32) + t%4 for step s,
// element t).  Samples 0..31 are lanes 0..31's own; samples 32..63 belong to
// lanes 32..63 and reach the B operand of lanes 0..31 by a cross-half
// exchange.  Every lane of the wave must call it (the products are
// wave-wide).
typedef _Float16 mlp_half8 __attribute__((ext_vector_type(8)));
typedef float mlp_f32x16 __attribute__((ext_vector_type(16)));

struct MlpFrags {
    mlp_half8 w1;      // first-layer A operand: hidden lane%32, inputs 8(lane/32) + t (bias at input 6)
    mlp_half8 w2[2];   // second-layer A operands of the two K steps
};

// b2 (32), w3 (32), b3: the output-layer constants a block keeps in LDS
constexpr int kMlpTail = 65;

__device__ __forceinline__ void mlp_tail_load(const float* __restrict__ P, float* __restrict__ tail)
{
    for (int q = threadIdx.x; q < kMlpTail; q += blockDim.x)
        tail[q] = (q < 32) ? P[kMlpB2 + q] : (q < 64) ? P[kMlpW3 + q - 32] : P[kMlpB3];
}

__device__ __forceinline__ void mlp_frags_load(const float* __restrict__ P, MlpFrags& M, int lane)
{
    const int r = lane & 31, g = lane >> 5;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float w = 0.0f;
        if (g == 0)
            w = (t < kMlpIn) ? P[kMlpW1 + kMlpIn * r + t] : (t == kMlpIn) ? P[kMlpB1 + r] : 0.0f;
        M.w1[t] = (_Float16)w;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int hid = 8 * (2 * s + t / 4) + 4 * g + (t % 4);
            M.w2[s][t] = (_Float16)P[kMlpW2 + kMlpHid * r + hid];
        }
}

// max(x, 0) rounded to binary16 (nearest, ties to even), widened exactly
__device__ __forceinline__ float half_relu(float x) { return (float)(_Float16)fmaxf(x, 0.0f); }

__device__ __forceinline__ float mlp_sigma_wave(const MlpFrags& M, const float* __restrict__ tail,
                                                const float (&f)[kMlpIn], int lane)
{
    const int g = lane >> 5;
    float fo[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
        fo[k] = __shfl_xor(f[k], 32);
    mlp_half8 x0, x1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const float a = (t < kMlpIn) ? f[t < kMlpIn ? t : 0] : (t == kMlpIn) ? 1.0f : 0.0f;
        const float b = (t < kMlpIn) ? fo[t < kMlpIn ? t : 0] : (t == kMlpIn) ? 1.0f : 0.0f;
        x0[t] = (_Float16)(g == 0 ? a : 0.0f);
        x1[t] = (_Float16)(g == 0 ? b : 0.0f);
    }
    mlp_f32x16 zero;
#pragma unroll
    for (int q = 0; q < 16; ++q)
        zero[q] = 0.0f;
    const mlp_f32x16 c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(M.w1, x0, zero, 0, 0, 0);
    const mlp_f32x16 c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(M.w1, x1, zero, 0, 0, 0);
    mlp_f32x16 d0 = zero, d1 = zero;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        mlp_half8 h0, h1;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            h0[t] = (_Float16)fmaxf(c0[8 * s + t], 0.0f);
            h1[t] = (_Float16)fmaxf(c1[8 * s + t], 0.0f);
        }
        d0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(M.w2[s], h0, d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(M.w2[s], h1, d1, 0, 0, 0);
    }
    float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 b2 = reinterpret_cast<const float4*>(tail)[2 * j + g];
        const float4 w3 = reinterpret_cast<const float4*>(tail + 32)[2 * j + g];
        p0 = fmaf(w3.x, half_relu(d0[4 * j + 0] + b2.x), p0);
        p0 = fmaf(w3.y, half_relu(d0[4 * j + 1] + b2.y), p0);
        p0 = fmaf(w3.z, half_relu(d0[4 * j + 2] + b2.z), p0);
        p0 = fmaf(w3.w, half_relu(d0[4 * j + 3] + b2.w), p0);
        p1 = fmaf(w3.x, half_relu(d1[4 * j + 0] + b2.x), p1);
        p1 = fmaf(w3.y, half_relu(d1[4 * j + 1] + b2.y), p1);
        p1 = fmaf(w3.z, half_relu(d1[4 * j + 2] + b2.z), p1);
        p1 = fmaf(w3.w, half_relu(d1[4 * j + 3] + b2.w), p1);
    }
    p0 += __shfl_xor(p0, 32);
    p1 += __shfl_xor(p1, 32);
    const float z = (g == 0 ? p0 : p1) + tail[64];
    return 1.0f / (1.0f + expf(-z));
}

}  // namespace pg
