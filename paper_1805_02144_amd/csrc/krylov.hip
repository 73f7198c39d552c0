// Vector kernels of phipm_simul_iom2 (Alg. 1): the IOM2 two-term update
// with the norm that yields h_{j+1,j}, the w_j recurrence when no product is
// needed, the substep combination y_{k+1} (eq. 3.17), input norms, and stage
// linear combinations of the schemes.  Reductions are deterministic
// (partials summed in block order by the consuming kernel).
#include "column.h"
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

constexpr int kRedBlock = 512;   // threads per block of the element-wise reducing kernels

inline int grid_elems(int n) {
    int g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return g > 4096 ? 4096 : g;
}

constexpr int kMaxLin = 6;

struct LinArgs {
    int k;
    const double *vec[kMaxLin];
    double c[kMaxLin];
};

__global__ void __launch_bounds__(kBlock) k_lincomb(int n4, double *__restrict__ out, LinArgs a) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxLin; ++k)
            if (k < a.k) acc += a.c[k] * a.vec[k][i];
        out[i] = acc;
    }
}

struct LinDevArgs {
    int k;
    const double *vec[kPmax + 1];
    const double *coef[kPmax + 1];
};

template <bool NORM>
__global__ void __launch_bounds__(kRedBlock) k_lincomb_dev(int n4, double *__restrict__ out,
                                                           LinDevArgs a, double *nrm_out) {
    __shared__ double lds[16];
    double c[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) c[k] = (k < a.k) ? *a.coef[k] : 0.0;
    double r = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k <= kPmax; ++k)
            if (k < a.k) acc += c[k] * a.vec[k][i];
        out[i] = acc;
        if (NORM) r += acc * acc;
    }
    if (!NORM) return;
    double v[1] = {r};
    block_sum_all<1>(v, lds);
    put_partials<1>(v, nrm_out);
}

// IOM2 update of column j (classical two-term Gram-Schmidt) and its norm.
__global__ void __launch_bounds__(kRedBlock) k_iom2_update(int n4, int j, double *__restrict__ w,
                                                           const double *__restrict__ rj,
                                                           const double *__restrict__ rjm1,
                                                           PhiCtl *ctl, const double *nrm_in,
                                                           int np_nrm, const double *dot_in,
                                                           int np_dot, double *nrm_out) {
    __shared__ double lds[64];
    // a new basis (j = 0) starts fresh; later columns stop after a breakdown
    if (j > 0 && (ctl->brk != 0 || ctl->beta_zero)) return;
    double nn[1], dd[2];
    sum_partials<1>(nn, nrm_in, np_nrm, lds);
    sum_partials<2>(dd, dot_in, np_dot, lds);
    const bool writer = blockIdx.x == 0 && threadIdx.x == 0;
    const ColumnScale cs = finalize_column(ctl, j, nn[0], writer, lds);
    if (cs.stop) return;
    const double sj = cs.sigma;
    const double sm = j > 0 ? ctl->sigma[j - 1] : 0.0;
    const double hjj = sj * sj * dd[0];
    const double hmj = j > 0 ? sj * sm * dd[1] : 0.0;
    if (writer) {
        ctl->H[j * kMmax + j] = hjj;
        if (j > 0) ctl->H[(j - 1) * kMmax + j] = hmj;
    }
    const double cj = hjj * sj;
    const double cm = hmj * sm;
    double r = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double x = sj * w[i] - cj * rj[i];
        if (j > 0) x -= cm * rjm1[i];
        w[i] = x;
        r += x * x;
    }
    double v[1] = {r};
    block_sum_all<1>(v, lds);
    put_partials<1>(v, nrm_out);
}

struct CombArgs {
    int p, meff, corr;
    const double *w[kPmax];   // w_0..w_{p-1}, nullptr = zero (skipped)
    const double *V;          // raw basis, vectors of length n4
};

__global__ void __launch_bounds__(kBlock) k_combine(int n4, double *__restrict__ y, CombArgs a,
                                                    const PhiCtl *__restrict__ ctl) {
    __shared__ double cf[kPmax + kMmax + 2];
    for (int k = threadIdx.x; k < kPmax + kMmax + 2; k += blockDim.x) cf[k] = ctl->ycoef[k];
    __syncthreads();
    const int nb = a.meff + (a.corr ? 1 : 0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < a.p; ++j)
            if (a.w[j]) acc += cf[j] * a.w[j][i];
        const double *vb = a.V + i;
        for (int k = 0; k < nb; ++k) acc += cf[a.p + k] * vb[(size_t)k * n4];
        y[i] = acc;
    }
}

struct NormArgs {
    int nv;
    const double *vec[kPmax + 1];
};

__global__ void __launch_bounds__(kRedBlock) k_norms(int n4, NormArgs a, double *parts) {
    __shared__ double lds[16 * (kPmax + 1)];
    double r[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) r[k] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k <= kPmax; ++k) {
            if (k < a.nv) {
                const double v = a.vec[k][i];
                r[k] += v * v;
            }
        }
    }
    block_sum_all<kPmax + 1>(r, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < a.nv; ++k) parts[blockIdx.x * a.nv + k] = r[k];
}

__global__ void __launch_bounds__(kBlock) k_phi_init(PhiCtl *c, int m0, double tau0,
                                                     double tol_rel, const double *parts, int np,
                                                     int nv, double *vn2) {
    __shared__ double lds[16 * (kPmax + 1)];
    double tot[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < np; b += blockDim.x)
        for (int k = 0; k < nv; ++k) tot[k] += parts[b * nv + k];
    block_sum_all<kPmax + 1>(tot, lds);
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nv; ++k) {
        vn2[k] = tot[k];
        const double r = sqrt(tot[k]);
        s = r > s ? r : s;
    }
    c->tol_abs = tol_rel * s;
    c->t = 0.0;
    c->tau = tau0;
    c->m = m0;
    c->q = (m0 / 4.0 > 1.0) ? m0 / 4.0 : 1.0;
    c->kappa = 2.0;
    c->have_prev = 0;
    c->prev_m = 0;
    c->prev_tau = 0.0;
    c->prev_omega = 0.0;
    c->rec_coef[0] = 1.0;
    for (int l = 1; l <= kPmax; ++l) c->rec_coef[l] = 0.0;
    c->brk = 0;
    c->beta_zero = 0;
    c->dec.status = 0;
}

__global__ void k_set_tout(PhiCtl *c, double t_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) c->t_out = t_out;
}

}  // namespace

void launch_lincomb(int n4, double *out, int k, const double *const *vec, const double *c,
                    hipStream_t s) {
    LinArgs a{};
    a.k = k;
    for (int i = 0; i < k && i < kMaxLin; ++i) {
        a.vec[i] = vec[i];
        a.c[i] = c[i];
    }
    hipLaunchKernelGGL(k_lincomb, dim3(grid_elems(n4)), dim3(kBlock), 0, s, n4, out, a);
}

int launch_lincomb_dev(int n, double *out, int k, const double *const *vec,
                       const double *const *coef, double *nrm_out, hipStream_t s) {
    LinDevArgs a{};
    a.k = k;
    for (int i = 0; i < k && i <= kPmax; ++i) {
        a.vec[i] = vec[i];
        a.coef[i] = coef[i];
    }
    const int n4 = 4 * n;
    const int grid = red_grid(n4, kRedBlock);
    if (nrm_out)
        hipLaunchKernelGGL(k_lincomb_dev<true>, dim3(grid), dim3(kRedBlock), 0, s, n4, out, a,
                           nrm_out);
    else
        hipLaunchKernelGGL(k_lincomb_dev<false>, dim3(grid), dim3(kRedBlock), 0, s, n4, out, a,
                           nrm_out);
    return grid;
}

int launch_iom2_update(int n, int j, double *rjp1, const double *rj, const double *rjm1,
                       PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                       int np_dot, double *nrm_out, hipStream_t s) {
    const int n4 = 4 * n;
    const int grid = red_grid(n4, kRedBlock);
    hipLaunchKernelGGL(k_iom2_update, dim3(grid), dim3(kRedBlock), 0, s, n4, j, rjp1, rj, rjm1,
                       ctl, nrm_in, np_nrm, dot_in, np_dot, nrm_out);
    return grid;
}

void launch_combine(int n4, double *y, int p, const double *const *w, const int *wzero,
                    const double *V, int meff, int corr, PhiCtl *ctl, hipStream_t s) {
    CombArgs a{};
    a.p = p;
    a.meff = meff;
    a.corr = corr;
    for (int j = 0; j < p; ++j) a.w[j] = wzero[j] ? nullptr : w[j];
    a.V = V;
    hipLaunchKernelGGL(k_combine, dim3(grid_elems(n4)), dim3(kBlock), 0, s, n4, y, a, ctl);
}

int launch_norms(int n, int nv, const double *const *vec, double *parts, hipStream_t s) {
    NormArgs a{};
    a.nv = nv;
    for (int k = 0; k < nv && k <= kPmax; ++k) a.vec[k] = vec[k];
    const int grid = red_grid(4 * n, kRedBlock);
    hipLaunchKernelGGL(k_norms, dim3(grid), dim3(kRedBlock), 0, s, 4 * n, a, parts);
    return grid;
}

void launch_phi_init(PhiCtl *ctl, int m0, double tau0, double tol_rel, const double *parts,
                     int np, int nv, double *vnorm2_out, hipStream_t s) {
    hipLaunchKernelGGL(k_phi_init, dim3(1), dim3(kBlock), 0, s, ctl, m0, tau0, tol_rel, parts, np,
                       nv, vnorm2_out);
}

void launch_set_tout(PhiCtl *ctl, double t_out, hipStream_t s) {
    hipLaunchKernelGGL(k_set_tout, dim3(1), dim3(64), 0, s, ctl, t_out);
}

}  // namespace xrb
