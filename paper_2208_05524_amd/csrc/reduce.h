// Deterministic workgroup reductions (fixed tree order, no atomics).
#pragma once

#include <hip/hip_runtime.h>

namespace vesis {
namespace {

constexpr int RED_WG = 256;

// Sum of v over the 256 lanes of the workgroup, identical on every run.
// Every lane must call it; the result is returned to all lanes.
template <typename T>
__device__ inline T block_sum(T v, T* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = RED_WG / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

// out[k] = sum over blocks b of partial[b * K + k], k < K, in block order
// chunks handled by fixed lanes, then a fixed tree.
template <typename T, int K>
__global__ __launch_bounds__(RED_WG) void reduce_partials(const T* partial, int nblocks, T* out) {
    __shared__ T sh[RED_WG];
    for (int k = 0; k < K; ++k) {
        T s = 0;
        for (int i = threadIdx.x; i < nblocks; i += RED_WG) s += partial[(int64_t)i * K + k];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[k] = s;
    }
}

}  // namespace
}  // namespace vesis
