// Deterministic reductions without floating-point atomics or fences.
//
// A producing kernel writes one partial per block (fixed in-block order).
// The consuming kernel -- the next one on the stream, so the kernel boundary
// makes the partials visible -- sums them in block order; every block of the
// consumer that needs the total computes it redundantly and bitwise
// identically.  (A device-scope fence per block, the usual "last block"
// pattern, costs an L2 write-back per block on a multi-XCD part.)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xrb_internal.h"

namespace xrb {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;  // valid in lane 0
}

// Sums NV values over the block (blockDim.x a multiple of 64, <= 1024);
// the result is returned in every thread.  lds must hold 16*NV doubles.
template <int NV>
__device__ inline void block_sum_all(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[wid * NV + k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

// Write this block's partials (thread 0 after block_sum_all); parts is the
// calling member's buffer.
template <int NV>
__device__ inline void put_partials(const double (&v)[NV], double *parts) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) parts[blockIdx.x * NV + k] = v[k];
    }
}

// Total of partials written by a previous kernel: fixed strided slices per
// thread, then block_sum_all.  Result in every thread.
template <int NV>
__device__ inline void sum_partials(double (&tot)[NV], const double *parts, int np, double *lds) {
#pragma unroll
    for (int k = 0; k < NV; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < np; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] += parts[b * NV + k];
    block_sum_all<NV>(tot, lds);
}

}  // namespace xrb
