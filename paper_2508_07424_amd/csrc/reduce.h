// Deterministic block reductions (wave64 butterflies, then a fixed-order sum
// over the waves of the block).  Each block writes its partial sums to
// partials[v * stride + block]; the consumer adds the blocks with
// block_sum_all, in a fixed order, so results are bitwise reproducible for a
// fixed launch shape.
#pragma once
#include <hip/hip_runtime.h>

namespace mirve {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum NV per-thread values over the block; thread 0 stores value i at
// partials[i * stride + bid].
template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double* partials, long long stride,
                                       int bid) {
    __shared__ double sh[NV][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[i][wid] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[i][w];
            partials[i * stride + bid] = s;
        }
    }
}

__device__ inline void block_max_store(double v, double* partials, int bid) {
    __shared__ double sh[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_max(v);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        double m = sh[0];
        for (int w = 1; w < nw; ++w) m = fmax(m, sh[w]);
        partials[bid] = m;
    }
}

// Fixed-order sum of NV arrays of n partials (array i at p[i * stride]) by
// the whole block; every thread of every block of a launch gets the same
// bits (the xor butterfly gives all lanes the same value, since IEEE
// addition is commutative).  Contains barriers: call from uniform control
// flow.
template <int NV>
__device__ inline void block_sum_all(const double* p, long long stride, int n, double (&out)[NV]) {
    __shared__ double sh[NV][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int k = threadIdx.x; k < n; k += blockDim.x) s += p[i * stride + k];
        s = wave_sum(s);
        if (lane == 0) sh[i][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[i][w];
        out[i] = s;
    }
    __syncthreads();
}

}  // namespace mirve
