// Deterministic block and grid reductions (fixed summation order, no
// floating-point atomics).  A grid reduction writes one partial per block;
// the last block to arrive (integer ticket) sums the partials in block order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xrb {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;  // valid in lane 0
}

// Sums NV values over a 256-thread block; result valid in thread 0.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *lds /* >= 4*NV */) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[wid * NV + k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            v[k] = ((lds[k] + lds[NV + k]) + lds[2 * NV + k]) + lds[3 * NV + k];
    }
}

__device__ inline double load_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this block's NV partials; returns true in every thread of the last
// block to arrive (which then owns the final sum).  Thread 0 must hold the
// block sums in v.
template <int NV>
__device__ inline bool grid_arrive(const double (&v)[NV], double *partials, uint32_t *counter) {
    __shared__ int last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) partials[blockIdx.x * NV + k] = v[k];
        __threadfence();
        uint32_t t = atomicAdd(counter, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// In the last block: total[k] = sum_b partials[b*NV+k], summed by a fixed
// tree (each thread a fixed strided slice, then block_sum).  Result in
// thread 0.  Resets the ticket counter.
template <int NV>
__device__ inline void grid_finish(double (&tot)[NV], const double *partials, uint32_t *counter,
                                   double *lds) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] += load_coherent(partials + b * NV + k);
    __syncthreads();
    block_sum<NV>(tot, lds);
    if (threadIdx.x == 0) *counter = 0u;
}

}  // namespace xrb
