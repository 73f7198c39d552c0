// Finalisation of one IOM2 column from the squared norm of the raw vector
// R_j that the previous kernel produced (Alg. 1, step 2(i)): j = 0 gives
// beta = ||w_p|| and the scale of v_1 = w_p / beta; j >= 1 gives
// h_{j,j-1} = ||R_j|| and the scale of v_{j+1}, or a happy breakdown when
// h_{j,j-1} <= 1e-14 ||H||_1 of the leading j x j block.  H is tridiagonal
// (orthogonalisation length 2), so column q of that block sums
// |h_{q-1,q}| + |h_{q,q}| + |h_{q+1,q}| (the last only when q+1 < j).
// Every thread of the block must call it; all get the same result, and
// only the thread passing write = true stores it.
#pragma once
#include "xrb_internal.h"

namespace xrb {

struct ColumnScale {
    double sigma;   // scale of R_j (0 when the process stops)
    int stop;       // beta == 0 or breakdown at this column
};

// max over the block of a non-negative value; lds >= 16 doubles
__device__ inline double block_max(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(v, off, 64);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = lds[w] > r ? lds[w] : r;
    __syncthreads();
    return r;
}

// |column q| of the leading j x j block of H for q = threadIdx.x (0 for
// threads past it); its block maximum is the ||H||_1 of the breakdown test.
__device__ inline double column_abs_sum(const PhiCtl *c, int j) {
    const int q = threadIdx.x;
    double cs = 0.0;
    if (q < j) {
        if (q > 0) cs = fabs(c->H[(q - 1) * kMmax + q]);
        cs += fabs(c->H[q * kMmax + q]);
        if (q + 1 < j) cs += fabs(c->H[(q + 1) * kMmax + q]);
    }
    return cs;
}

// Column finalisation given ss = ||R_j||^2 and, for j >= 1, bn = ||H||_1 of
// the leading j x j block.
__device__ inline ColumnScale finalize_column_bn(PhiCtl *c, int j, double ss, double bn,
                                                 bool write) {
    const double h = sqrt(ss);
    if (j == 0) {
        if (write) {
            c->beta = h;
            c->beta_zero = (h == 0.0) ? 1 : 0;
            c->sigma[0] = h > 0.0 ? 1.0 / h : 0.0;
            c->brk = 0;
            if (h != h) c->dec.status = XRB_ENAN;
        }
        return {h > 0.0 ? 1.0 / h : 0.0, !(h > 0.0)};
    }
    if (!(h > 1e-14 * bn)) {
        if (write) {
            if (h != h) c->dec.status = XRB_ENAN;
            c->H[j * kMmax + j - 1] = 0.0;
            c->sigma[j] = 0.0;
            c->brk = j;
        }
        return {0.0, 1};
    }
    if (write) {
        c->H[j * kMmax + j - 1] = h;
        c->sigma[j] = 1.0 / h;
    }
    return {1.0 / h, 0};
}

__device__ inline ColumnScale finalize_column(PhiCtl *c, int j, double ss, bool write,
                                              double *lds) {
    const double bn = j > 0 ? block_max(column_abs_sum(c, j), lds) : 0.0;
    return finalize_column_bn(c, j, ss, bn, write);
}

}  // namespace xrb
