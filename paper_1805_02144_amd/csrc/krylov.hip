// Vector kernels of phipm_simul_iom2 (Alg. 1): the IOM2 two-term update
// with the norm that yields h_{j+1,j}, the w_j recurrence when no product is
// needed, the substep combination y_{k+1} (eq. 3.17) and stage linear
// combinations of the schemes.  All reductions are deterministic.
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

inline int grid_capped(int n) {
    int g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return g > kMaxBlocks ? kMaxBlocks : g;
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
__global__ void __launch_bounds__(kBlock) k_lincomb_dev(int n4, double *__restrict__ out,
                                                        LinDevArgs a, PhiCtl *ctl,
                                                        double *partials) {
    __shared__ double lds[8];
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
    block_sum<1>(v, lds);
    if (!grid_arrive<1>(v, partials, &ctl->counters[1])) return;
    double tot[1];
    grid_finish<1>(tot, partials, &ctl->counters[1], lds);
    if (threadIdx.x == 0) {
        const double beta = sqrt(tot[0]);
        ctl->beta = beta;
        ctl->beta_zero = (beta == 0.0) ? 1 : 0;
        ctl->sigma[0] = beta > 0.0 ? 1.0 / beta : 0.0;
        ctl->brk = 0;
    }
}

// IOM2 update of column j (classical two-term Gram-Schmidt) and its norm.
__global__ void __launch_bounds__(kBlock) k_iom2_update(int n4, int j, double *__restrict__ w,
                                                        const double *__restrict__ rj,
                                                        const double *__restrict__ rjm1,
                                                        PhiCtl *ctl, double *partials) {
    __shared__ double lds[8];
    if (ctl->brk != 0 || ctl->beta_zero) return;
    const double cj = ctl->H[j * kMmax + j] * ctl->sigma[j];
    const double cm = (j > 0) ? ctl->H[(j - 1) * kMmax + j] * ctl->sigma[j - 1] : 0.0;
    double r = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double x = w[i] - cj * rj[i];
        if (j > 0) x -= cm * rjm1[i];
        w[i] = x;
        r += x * x;
    }
    double v[1] = {r};
    block_sum<1>(v, lds);
    if (!grid_arrive<1>(v, partials, &ctl->counters[2])) return;
    double tot[1];
    grid_finish<1>(tot, partials, &ctl->counters[2], lds);
    if (threadIdx.x == 0) {
        const double hn = sqrt(tot[0]);
        if (hn != hn) ctl->dec.status = XRB_ENAN;
        // breakdown when h_{j+1,j} <= 1e-14 * ||H_j||_1 (square leading block)
        double bn = 0.0;
        for (int c = 0; c <= j; ++c) {
            double cs = 0.0;
            for (int rr = 0; rr <= j; ++rr) cs += fabs(ctl->H[rr * kMmax + c]);
            bn = cs > bn ? cs : bn;
        }
        if (!(hn > 1e-14 * bn)) {
            ctl->H[(j + 1) * kMmax + j] = 0.0;
            ctl->sigma[j + 1] = 0.0;
            ctl->brk = j + 1;
        } else {
            ctl->H[(j + 1) * kMmax + j] = hn;
            ctl->sigma[j + 1] = 1.0 / hn;
        }
    }
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

__global__ void __launch_bounds__(kBlock) k_norm2(int n4, const double *__restrict__ x,
                                                  double *out, double *partials,
                                                  uint32_t *counter) {
    __shared__ double lds[8];
    double r = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x)
        r += x[i] * x[i];
    double v[1] = {r};
    block_sum<1>(v, lds);
    if (!grid_arrive<1>(v, partials, counter)) return;
    double tot[1];
    grid_finish<1>(tot, partials, counter, lds);
    if (threadIdx.x == 0) *out = tot[0];
}

__global__ void k_phi_init(PhiCtl *c, int m0, double tau0, double tol_rel, const double *vn2,
                           int nv) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nv; ++k) {
        double r = sqrt(vn2[k]);
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
    hipLaunchKernelGGL(k_lincomb, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4, out, a);
}

void launch_lincomb_dev(int n4, double *out, int k, const double *const *vec,
                        const double *const *coef, PhiCtl *ctl, double *partials, int norm,
                        hipStream_t s) {
    LinDevArgs a{};
    a.k = k;
    for (int i = 0; i < k && i <= kPmax; ++i) {
        a.vec[i] = vec[i];
        a.coef[i] = coef[i];
    }
    if (norm)
        hipLaunchKernelGGL(k_lincomb_dev<true>, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4,
                           out, a, ctl, partials);
    else
        hipLaunchKernelGGL(k_lincomb_dev<false>, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4,
                           out, a, ctl, partials);
}

void launch_iom2_update(int n4, int j, double *rjp1, const double *rj, const double *rjm1,
                        PhiCtl *ctl, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_iom2_update, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4, j, rjp1, rj,
                       rjm1, ctl, partials);
}

void launch_combine(int n4, double *y, int p, const double *const *w, const int *wzero,
                    const double *V, int meff, int corr, PhiCtl *ctl, hipStream_t s) {
    CombArgs a{};
    a.p = p;
    a.meff = meff;
    a.corr = corr;
    for (int j = 0; j < p; ++j) a.w[j] = wzero[j] ? nullptr : w[j];
    a.V = V;
    hipLaunchKernelGGL(k_combine, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4, y, a, ctl);
}

void launch_norm2(int n4, const double *x, double *out, double *partials, uint32_t *counter,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, dim3(grid_capped(n4)), dim3(kBlock), 0, s, n4, x, out, partials,
                       counter);
}

void launch_phi_init(PhiCtl *ctl, int m0, double tau0, double tol_rel, const double *vnorm2,
                     int nv, hipStream_t s) {
    hipLaunchKernelGGL(k_phi_init, dim3(1), dim3(64), 0, s, ctl, m0, tau0, tol_rel, vnorm2, nv);
}

void launch_set_tout(PhiCtl *ctl, double t_out, hipStream_t s) {
    hipLaunchKernelGGL(k_set_tout, dim3(1), dim3(64), 0, s, ctl, t_out);
}

}  // namespace xrb
