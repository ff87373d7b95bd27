// Small device helpers shared by the association and solve kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace pg {

// upper-triangle index of (a, b), a <= b, in an n x n symmetric matrix
__host__ __device__ constexpr int upper_index(int a, int b, int n) { return a * n - a * (a - 1) / 2 + (b - a); }

// packed lower-triangle index of (i, j), i >= j
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename T>
__device__ __forceinline__ T ld_global(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

typedef float pg_f4v __attribute__((ext_vector_type(4)));
template <>
__device__ __forceinline__ float4 ld_global<float4>(const float4* p)
{
    const pg_f4v v = *(const __attribute__((address_space(1))) pg_f4v*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Stores through global-address pointers (pointers held in C++ structures are
// generic): global stores, which LDS waits do not count.
template <typename T>
__device__ __forceinline__ void st_global(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

template <>
__device__ __forceinline__ void st_global<float4>(float4* p, float4 v)
{
    const pg_f4v w = {v.x, v.y, v.z, v.w};
    *(__attribute__((address_space(1))) pg_f4v*)p = w;
}

}  // namespace pg
