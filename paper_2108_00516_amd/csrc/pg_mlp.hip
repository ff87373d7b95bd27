// Training and inference kernels of the learned correspondence weighting
// network, and the C ABI of its trainer (pg_mlp_*).
//
// Loss: mean binary cross-entropy of sigmoid(logit) against 0/1 labels, over
// a batch resident in device memory.  Gradient: per block of 64 samples, one
// thread per sample runs the forward and backward pass and leaves its
// activations and deltas in LDS; the block then forms every parameter's sum
// over its 64 samples in a fixed order (FP32), and a second kernel adds the
// block sums in block order in FP64 and divides by the batch size.  The
// result does not depend on scheduling.  Adam keeps FP32 master parameters
// and moments and writes an fp16 copy for the association kernels.
#include "pg_mlp.hpp"
#include "posegraph.h"

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>

namespace pg {
namespace {

constexpr int kTrainSamples = 64;               // samples (threads) per block
constexpr int kGradSlots = kMlpParams + 1;      // parameter sums, then the loss sum
constexpr int kLdsStride = 33;                  // row stride of the LDS tables

// LDS tables, one row per sample: X holds x (cols 0..5), 1 (col 6), the
// sample's loss (col 7) and dloss/dlogit (col 8).
struct TrainLds {
    float X[kTrainSamples][kLdsStride];
    float H1[kTrainSamples][kLdsStride];
    float H2[kTrainSamples][kLdsStride];
    float D1[kTrainSamples][kLdsStride];
    float D2[kTrainSamples][kLdsStride];
};

__global__ __launch_bounds__(kTrainSamples) void mlp_grad_kernel(const float* __restrict__ x,
                                                                 const float* __restrict__ labels, int n,
                                                                 const float* __restrict__ P,
                                                                 float* __restrict__ part)
{
    __shared__ TrainLds L;
    const int t = threadIdx.x;
    const int s = blockIdx.x * kTrainSamples + t;
    const bool live = s < n;
    float xi[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
        xi[k] = live ? x[(size_t)kMlpIn * s + k] : 0.0f;
    // forward
    float a1[kMlpHid];
#pragma unroll
    for (int o = 0; o < kMlpHid; ++o) {
        float a = P[kMlpB1 + o];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k)
            a = fmaf(P[kMlpW1 + kMlpIn * o + k], xi[k], a);
        a1[o] = a;
        L.H1[t][o] = fmaxf(a, 0.0f);
    }
    float z = P[kMlpB3];
    unsigned int act2 = 0;   // bit o: a2[o] > 0
    for (int o = 0; o < kMlpHid; ++o) {
        float a = P[kMlpB2 + o];
#pragma unroll
        for (int k = 0; k < kMlpHid; ++k)
            a = fmaf(P[kMlpW2 + kMlpHid * o + k], fmaxf(a1[k], 0.0f), a);
        const float h = fmaxf(a, 0.0f);
        L.H2[t][o] = live ? h : 0.0f;
        act2 |= (a > 0.0f ? 1u : 0u) << o;
        z = fmaf(P[kMlpW3 + o], h, z);
    }
    // loss log(1 + e^z) - y z, and its derivative sigmoid(z) - y
    const float y = live ? labels[s] : 0.0f;
    const float sp = (z > 0.0f) ? z + log1pf(expf(-z)) : log1pf(expf(z));
    const float dz = live ? 1.0f / (1.0f + expf(-z)) - y : 0.0f;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
        L.X[t][k] = xi[k];
    L.X[t][6] = 1.0f;
    L.X[t][7] = live ? sp - y * z : 0.0f;
    L.X[t][8] = dz;
    // backward
    float d2[kMlpHid];
#pragma unroll
    for (int o = 0; o < kMlpHid; ++o) {
        d2[o] = ((act2 >> o) & 1u) ? dz * P[kMlpW3 + o] : 0.0f;
        L.D2[t][o] = d2[o];
    }
    for (int k = 0; k < kMlpHid; ++k) {
        float acc = 0.0f;
#pragma unroll
        for (int o = 0; o < kMlpHid; ++o)
            acc = fmaf(P[kMlpW2 + kMlpHid * o + k], d2[o], acc);
        L.D1[t][k] = (live && a1[k] > 0.0f) ? acc : 0.0f;
    }
    __syncthreads();
    // parameter sums over the block's samples: slot q = sum_s U[s][u] V[s][v]
    float* __restrict__ out = part + (size_t)blockIdx.x * kGradSlots;
    for (int q = t; q < kGradSlots; q += kTrainSamples) {
        const float* U;
        const float* Vv;
        if (q < kMlpB1) {                     // W1[o][k]: d1[o] x[k]
            U = &L.D1[0][q / kMlpIn];
            Vv = &L.X[0][q % kMlpIn];
        } else if (q < kMlpW2) {              // b1[o]: d1[o]
            U = &L.D1[0][q - kMlpB1];
            Vv = &L.X[0][6];
        } else if (q < kMlpB2) {              // W2[o][k]: d2[o] h1[k]
            const int r = q - kMlpW2;
            U = &L.D2[0][r / kMlpHid];
            Vv = &L.H1[0][r % kMlpHid];
        } else if (q < kMlpW3) {              // b2[o]: d2[o]
            U = &L.D2[0][q - kMlpB2];
            Vv = &L.X[0][6];
        } else if (q < kMlpB3) {              // W3[o]: dz h2[o]
            U = &L.X[0][8];
            Vv = &L.H2[0][q - kMlpW3];
        } else if (q == kMlpB3) {             // b3: dz
            U = &L.X[0][8];
            Vv = &L.X[0][6];
        } else {                              // loss
            U = &L.X[0][7];
            Vv = &L.X[0][6];
        }
        float acc = 0.0f;
#pragma unroll 8
        for (int r = 0; r < kTrainSamples; ++r)
            acc = fmaf(U[r * kLdsStride], Vv[r * kLdsStride], acc);
        out[q] = acc;
    }
}

// out[q] = (sum over blocks, in block order, FP64) / n
__global__ void mlp_grad_reduce_kernel(const float* __restrict__ part, int n_blocks, int n,
                                       double* __restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kGradSlots)
        return;
    double s = 0.0;
    for (int b = 0; b < n_blocks; ++b)
        s += (double)part[(size_t)b * kGradSlots + q];
    out[q] = s / (double)n;
}

// Adam (bias-corrected: c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t))
__global__ void mlp_adam_kernel(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                                __half* __restrict__ p16, const double* __restrict__ grad, float lr, float beta1,
                                float beta2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams)
        return;
    const float g = (float)grad[q];
    const float mq = fmaf(beta1, m[q], (1.0f - beta1) * g);
    const float vq = fmaf(beta2, v[q], (1.0f - beta2) * g * g);
    m[q] = mq;
    v[q] = vq;
    const float p = P[q] - lr * (mq * c1) / (sqrtf(vq * c2) + eps);
    P[q] = p;
    p16[q] = __float2half_rn(p);
}

__global__ void mlp_to_half_kernel(const float* __restrict__ P, __half* __restrict__ p16)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < kMlpParams)
        p16[q] = __float2half_rn(P[q]);
}

__global__ void mlp_forward_kernel(const float* __restrict__ x, int n, const float* __restrict__ P,
                                   float* __restrict__ y)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    float f[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
        f[k] = x[(size_t)kMlpIn * s + k];
    y[s] = mlp_sigma(P, f);
}

bool device_ptr(const void* p)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

std::string g_mlp_create_error;

}  // namespace
}  // namespace pg

using namespace pg;

struct pg_mlp {
    hipStream_t stream = nullptr;
    int device = 0;
    int max_samples = 0;
    int step = 0;
    std::string err;
    float* P = nullptr;          // FP32 master parameters
    float* m = nullptr;          // Adam moments
    float* v = nullptr;
    __half* p16 = nullptr;       // fp16 copy
    double* out = nullptr;       // gradient and loss of the last batch (kGradSlots)
    float* part = nullptr;       // per-block sums
    double* h_out = nullptr;     // pinned readback
};

namespace {

pg_status mlp_fail(pg_mlp* t, pg_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (t)
        t->err = buf;
    else
        g_mlp_create_error = buf;
    return s;
}

#define MLP_HIP(t, call)                                                                                 \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return mlp_fail((t), e_ == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP, "%s: %s", \
                            #call, hipGetErrorString(e_));                                               \
    } while (0)

pg_status check_batch(pg_mlp* t, const float* x, const float* labels, int n, bool need_labels)
{
    if (!t)
        return PG_ERR_INVALID_ARG;
    if (n < 1 || n > t->max_samples)
        return mlp_fail(t, PG_ERR_INVALID_ARG, "batch of %d samples outside 1..%d", n, t->max_samples);
    if (!x || !device_ptr(x))
        return mlp_fail(t, PG_ERR_INVALID_ARG, "features must be device memory");
    if (need_labels && (!labels || !device_ptr(labels)))
        return mlp_fail(t, PG_ERR_INVALID_ARG, "labels must be device memory");
    MLP_HIP(t, hipSetDevice(t->device));
    return PG_OK;
}

hipError_t enqueue_grad(pg_mlp* t, const float* x, const float* labels, int n)
{
    const int nb = (n + kTrainSamples - 1) / kTrainSamples;
    mlp_grad_kernel<<<nb, kTrainSamples, 0, t->stream>>>(x, labels, n, t->P, t->part);
    mlp_grad_reduce_kernel<<<(kGradSlots + 255) / 256, 256, 0, t->stream>>>(t->part, nb, n, t->out);
    return hipGetLastError();
}

}  // namespace

extern "C" {

pg_status pg_mlp_create(int max_samples, void* hip_stream, pg_mlp** out)
{
    if (!out)
        return mlp_fail(nullptr, PG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_samples < 1 || max_samples > (1 << 26))
        return mlp_fail(nullptr, PG_ERR_INVALID_ARG, "max_samples %d outside 1..2^26", max_samples);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return mlp_fail(nullptr, PG_ERR_NO_DEVICE, "no HIP device");
    }
    pg_mlp* t = new pg_mlp();
    t->stream = (hipStream_t)hip_stream;
    t->max_samples = max_samples;
    hipError_t e = hipGetDevice(&t->device);
    const size_t nb = (size_t)(max_samples + kTrainSamples - 1) / kTrainSamples;
    if (e == hipSuccess) e = hipMalloc(&t->P, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&t->m, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&t->v, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&t->p16, sizeof(__half) * kMlpParams);
    if (e == hipSuccess) e = hipMalloc(&t->out, sizeof(double) * kGradSlots);
    if (e == hipSuccess) e = hipMalloc(&t->part, sizeof(float) * kGradSlots * nb);
    if (e == hipSuccess) e = hipHostMalloc(&t->h_out, sizeof(double) * kGradSlots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(t->P, 0, sizeof(float) * kMlpParams, t->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->m, 0, sizeof(float) * kMlpParams, t->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->v, 0, sizeof(float) * kMlpParams, t->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->p16, 0, sizeof(__half) * kMlpParams, t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    if (e != hipSuccess) {
        pg_status s = mlp_fail(nullptr, e == hipErrorOutOfMemory ? PG_ERR_OUT_OF_MEMORY : PG_ERR_HIP,
                               "trainer allocation: %s", hipGetErrorString(e));
        pg_mlp_destroy(t);
        return s;
    }
    *out = t;
    return PG_OK;
}

void pg_mlp_destroy(pg_mlp* t)
{
    if (!t)
        return;
    (void)hipSetDevice(t->device);
    if (t->stream)
        (void)hipStreamSynchronize(t->stream);
    else
        (void)hipDeviceSynchronize();
    (void)hipFree(t->P);
    (void)hipFree(t->m);
    (void)hipFree(t->v);
    (void)hipFree(t->p16);
    (void)hipFree(t->out);
    (void)hipFree(t->part);
    if (t->h_out)
        (void)hipHostFree(t->h_out);
    delete t;
}

pg_status pg_mlp_set_params(pg_mlp* t, const float* params)
{
    if (!t)
        return PG_ERR_INVALID_ARG;
    if (!params)
        return mlp_fail(t, PG_ERR_INVALID_ARG, "params is NULL");
    MLP_HIP(t, hipSetDevice(t->device));
    MLP_HIP(t, hipMemcpyAsync(t->P, params, sizeof(float) * kMlpParams,
                              device_ptr(params) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, t->stream));
    MLP_HIP(t, hipMemsetAsync(t->m, 0, sizeof(float) * kMlpParams, t->stream));
    MLP_HIP(t, hipMemsetAsync(t->v, 0, sizeof(float) * kMlpParams, t->stream));
    mlp_to_half_kernel<<<(kMlpParams + 255) / 256, 256, 0, t->stream>>>(t->P, t->p16);
    MLP_HIP(t, hipGetLastError());
    MLP_HIP(t, hipStreamSynchronize(t->stream));
    t->step = 0;
    return PG_OK;
}

pg_status pg_mlp_get_params(pg_mlp* t, float* params_out, void* fp16_out)
{
    if (!t)
        return PG_ERR_INVALID_ARG;
    MLP_HIP(t, hipSetDevice(t->device));
    if (params_out)
        MLP_HIP(t, hipMemcpyAsync(params_out, t->P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, t->stream));
    if (fp16_out)
        MLP_HIP(t, hipMemcpyAsync(fp16_out, t->p16, sizeof(__half) * kMlpParams, hipMemcpyDeviceToHost, t->stream));
    MLP_HIP(t, hipStreamSynchronize(t->stream));
    return PG_OK;
}

pg_status pg_mlp_loss_grad(pg_mlp* t, const float* x, const float* labels, int n, double* loss_out,
                           double* grad_out)
{
    pg_status s = check_batch(t, x, labels, n, true);
    if (s != PG_OK)
        return s;
    MLP_HIP(t, enqueue_grad(t, x, labels, n));
    MLP_HIP(t, hipMemcpyAsync(t->h_out, t->out, sizeof(double) * kGradSlots, hipMemcpyDeviceToHost, t->stream));
    MLP_HIP(t, hipStreamSynchronize(t->stream));
    if (grad_out)
        for (int q = 0; q < kMlpParams; ++q)
            grad_out[q] = t->h_out[q];
    if (loss_out)
        *loss_out = t->h_out[kMlpParams];
    return PG_OK;
}

pg_status pg_mlp_adam_step(pg_mlp* t, const float* x, const float* labels, int n, double lr, double* loss_out)
{
    pg_status s = check_batch(t, x, labels, n, true);
    if (s != PG_OK)
        return s;
    if (!(lr > 0.0 && lr < 1.0))
        return mlp_fail(t, PG_ERR_INVALID_ARG, "learning rate %g outside (0, 1)", lr);
    const double b1 = 0.9, b2 = 0.999;
    const int step = t->step + 1;
    const double c1 = 1.0 / (1.0 - pow(b1, step)), c2 = 1.0 / (1.0 - pow(b2, step));
    MLP_HIP(t, enqueue_grad(t, x, labels, n));
    mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, t->stream>>>(t->P, t->m, t->v, t->p16, t->out, (float)lr,
                                                                      (float)b1, (float)b2, 1e-8f, (float)c1,
                                                                      (float)c2);
    MLP_HIP(t, hipGetLastError());
    t->step = step;
    if (loss_out) {
        // the loss of the batch at the parameters before the step
        MLP_HIP(t, hipMemcpyAsync(t->h_out + kMlpParams, t->out + kMlpParams, sizeof(double),
                                  hipMemcpyDeviceToHost, t->stream));
        MLP_HIP(t, hipStreamSynchronize(t->stream));
        *loss_out = t->h_out[kMlpParams];
    }
    return PG_OK;
}

pg_status pg_mlp_forward(pg_mlp* t, const float* x, int n, float* y)
{
    pg_status s = check_batch(t, x, nullptr, n, false);
    if (s != PG_OK)
        return s;
    if (!y || !device_ptr(y))
        return mlp_fail(t, PG_ERR_INVALID_ARG, "output must be device memory");
    mlp_forward_kernel<<<(n + 255) / 256, 256, 0, t->stream>>>(x, n, t->P, y);
    MLP_HIP(t, hipGetLastError());
    MLP_HIP(t, hipStreamSynchronize(t->stream));
    return PG_OK;
}

const char* pg_mlp_last_error(const pg_mlp* t)
{
    return t ? t->err.c_str() : g_mlp_create_error.c_str();
}

}  // extern "C"
