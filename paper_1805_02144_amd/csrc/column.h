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
#include "reduce.h"
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

// Coefficients of the IOM2 update of column j (classical two-term
// Gram-Schmidt, Alg. 1 step 2(i)): R_{j+1} = sj w - cj R_j - cm R_{j-1}.
struct IomCoef {
    double sj, cj, cm;
    int stop;   // beta == 0 or breakdown at this column: no update
};

// The update's prologue, in every block of the kernel that applies the
// update: ||R_j||^2 from the np_nrm norm partials, <w, R_j> and <w, R_{j-1}>
// from the np_dot dot partials (member mk's rows), and the largest column sum
// of H, all issued at once and reduced behind one barrier in the same order
// as separate block reductions would; then the column scale, and the H
// entries written by block 0's thread 0.  pro: 64 doubles of LDS.  Every
// thread of the block must call it.
__device__ inline IomCoef iom2_coefficients(PhiCtl *ctl, int j, int mk, const double *nrm_in,
                                            int np_nrm, const double *dot_in, int np_dot,
                                            double *pro) {
    double v[3] = {0.0, 0.0, 0.0};
    const double *nk = nrm_in + (size_t)mk * kPartStride;
    const double *dk = dot_in + (size_t)mk * kPartStride;
    for (int b = threadIdx.x; b < np_nrm; b += blockDim.x) v[0] += nk[b];
    for (int b = threadIdx.x; b < np_dot; b += blockDim.x) {
        v[1] += dk[2 * b];
        v[2] += dk[2 * b + 1];
    }
    double cm_ = j > 0 ? column_abs_sum(ctl, j) : 0.0;
    {
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = wave_sum(v[k]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(cm_, off, 64);
            cm_ = o > cm_ ? o : cm_;
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) pro[wid * 4 + k] = v[k];
            pro[wid * 4 + 3] = cm_;
        }
        __syncthreads();
        double t[3] = {0.0, 0.0, 0.0}, bn = 0.0;
        for (int q = 0; q < nw; ++q) {
#pragma unroll
            for (int k = 0; k < 3; ++k) t[k] += pro[q * 4 + k];
            bn = pro[q * 4 + 3] > bn ? pro[q * 4 + 3] : bn;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = t[k];
        cm_ = bn;
    }
    const bool writer = blockIdx.x == 0 && threadIdx.x == 0;
    const ColumnScale cs = finalize_column_bn(ctl, j, v[0], cm_, writer);
    if (cs.stop) return {0.0, 0.0, 0.0, 1};
    const double sj = cs.sigma;
    const double sm = j > 0 ? ctl->sigma[j - 1] : 0.0;
    const double hjj = sj * sj * v[1];
    const double hmj = j > 0 ? sj * sm * v[2] : 0.0;
    if (writer) {
        ctl->H[j * kMmax + j] = hjj;
        if (j > 0) ctl->H[(j - 1) * kMmax + j] = hmj;
    }
    return {sj, hjj * sj, hmj * sm, 0};
}

// One pair of R_{j+1} = sj w - cj R_j - cm R_{j-1} (R_{j-1} absent at j = 0),
// without contraction, so that every kernel applying it forms the same bits
__device__ inline double2 iom2_pair(const IomCoef &k, int j, double2 a, double2 b, double2 c) {
#pragma clang fp contract(off)
    double2 x;
    x.x = k.sj * a.x - k.cj * b.x;
    x.y = k.sj * a.y - k.cj * b.y;
    if (j > 0) {
        x.x -= k.cm * c.x;
        x.y -= k.cm * c.y;
    }
    return x;
}

}  // namespace xrb
