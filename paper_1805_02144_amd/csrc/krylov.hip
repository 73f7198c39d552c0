// Vector kernels of phipm_simul_iom2 (Alg. 1): the IOM2 two-term update
// with the norm that yields h_{j+1,j}, the w_j recurrence when no product is
// needed, the substep combination y_{k+1} (eq. 3.17), input norms, output
// copies and stage linear combinations of the schemes.  Reductions are
// deterministic (partials summed in block order by the consuming kernel).
// All kernels run over nm members (blockIdx.y), see Batch.
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
    unsigned dtmask;
    const double *vec[kMaxLin];
    double c[kMaxLin];
};

__global__ void __launch_bounds__(kBlock) k_lincomb(int n4, double *__restrict__ out, LinArgs a,
                                                    Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    double c[kMaxLin];
    const double *v[kMaxLin];
    const double dk = bt.dtk ? bt.dtk[mk] : 1.0;
#pragma unroll
    for (int k = 0; k < kMaxLin; ++k) {
        c[k] = ((a.dtmask >> k) & 1) ? a.c[k] * dk : a.c[k];
        v[k] = (k < a.k) ? member_ptr(a.vec[k], bt.ws, mk) : nullptr;
    }
    out = member_ptr(out, bt.ws, mk);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxLin; ++k)
            if (k < a.k) acc += c[k] * v[k][i];
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
                                                           LinDevArgs a, double *nrm_out,
                                                           Batch bt) {
    __shared__ double lds[16];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    double c[kPmax + 1];
    const double *v[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) {
        c[k] = (k < a.k) ? *ctl_field(a.coef[k], mk) : 0.0;
        v[k] = (k < a.k) ? member_ptr(a.vec[k], bt.ws, mk) : nullptr;
    }
    out = member_ptr(out, bt.ws, mk);
    double r = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k <= kPmax; ++k)
            if (k < a.k) acc += c[k] * v[k][i];
        out[i] = acc;
        if (NORM) r += acc * acc;
    }
    if (!NORM) return;
    double vv[1] = {r};
    block_sum_all<1>(vv, lds);
    put_partials<1>(vv, nrm_out + (size_t)mk * kPartStride);
}

// IOM2 update of column j (classical two-term Gram-Schmidt) and its norm.
// The body streams 16-byte pairs (n4 is even and every vector starts 16-byte
// aligned).  Latency shape: the thread's first kUpdPre pairs of w, R_j and
// R_{j-1} are requested before the prologue (the column scale needs the
// previous kernels' partials and H), and the prologue issues all its loads
// at once and reduces the three sums and the column maximum behind one
// barrier -- in the same order as separate block reductions would.
constexpr int kUpdPre = 4;

__global__ void __launch_bounds__(kRedBlock) k_iom2_update(int n4, int j, double *__restrict__ w,
                                                           const double *__restrict__ rj,
                                                           const double *__restrict__ rjm1,
                                                           PhiCtl *ctl0, const double *nrm_in,
                                                           int np_nrm, const double *dot_in,
                                                           int np_dot, double *nrm_out, Batch bt) {
    __shared__ double pro[16 * 4];
    __shared__ double lds[16];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    double2 *w2 = reinterpret_cast<double2 *>(member_ptr(w, bt.ws, mk));
    const double2 *r2 = reinterpret_cast<const double2 *>(member_ptr(rj, bt.ws, mk));
    const double2 *m2 = reinterpret_cast<const double2 *>(member_ptr(rjm1, bt.ws, mk));
    const int nv = n4 / 2;
    const int stride = gridDim.x * blockDim.x;
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    const double2 z2 = make_double2(0.0, 0.0);
    double2 pw[kUpdPre], pr[kUpdPre], pm[kUpdPre];
#pragma unroll
    for (int u = 0; u < kUpdPre; ++u) {
        const int i = i0 + u * stride;
        const bool in = i < nv;
        pw[u] = in ? w2[i] : z2;
        pr[u] = in ? r2[i] : z2;
        pm[u] = (in && j > 0) ? m2[i] : z2;
    }
    PhiCtl *ctl = ctl_member(ctl0, mk);
    // a new basis (j = 0) starts fresh; later columns stop after a breakdown
    if (j > 0 && (ctl->brk != 0 || ctl->beta_zero)) return;
    // prologue: ||R_j||^2, <w, R_j>, <w, R_{j-1}>, max column sum of H, scale
    const IomCoef kc = iom2_coefficients(ctl, j, mk, nrm_in, np_nrm, dot_in, np_dot, pro);
    if (kc.stop) return;
    double r = 0.0;
    auto upd = [&](double2 a, double2 b, double2 c) {
        const double2 x = iom2_pair(kc, j, a, b, c);
        r += x.x * x.x;
        r += x.y * x.y;
        return x;
    };
#pragma unroll
    for (int u = 0; u < kUpdPre; ++u) {
        const int i = i0 + u * stride;
        if (i < nv) w2[i] = upd(pw[u], pr[u], pm[u]);
    }
    for (int i = i0 + kUpdPre * stride; i < nv; i += stride)
        w2[i] = upd(w2[i], r2[i], j > 0 ? m2[i] : z2);
    double vv[1] = {r};
    block_sum_all<1>(vv, lds);
    put_partials<1>(vv, nrm_out + (size_t)mk * kPartStride);
}

struct CombArgs {
    int p;
    const double *w[kPmax];   // w_0..w_{p-1}, nullptr = zero (skipped)
    const double *V;          // raw basis, vectors of length n4
};

__global__ void __launch_bounds__(kBlock) k_combine(int n4, double *__restrict__ y, CombArgs a,
                                                    const PhiCtl *__restrict__ ctl0, Batch bt) {
    __shared__ double cf[kPmax + kMmax + 2];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const PhiCtl *ctl = ctl0 + mk;
    for (int k = threadIdx.x; k < kPmax + kMmax + 2; k += blockDim.x) cf[k] = ctl->ycoef[k];
    const int meff = ctl->dec.m_eff;
    __syncthreads();
    const int nb = meff > 0 ? meff + 1 : 0;
    y = member_ptr(y, bt.ws, mk);
    // per-member zero flags of w_j ride in the plan entry (bit j+1)
    const int zmask = bt.pred.plan ? (bt.pred.plan[kPlanW * mk + PF_COMB] >> 1) : 0;
    const double *w[kPmax];
#pragma unroll
    for (int j = 0; j < kPmax; ++j)
        w[j] = (j < a.p && !((zmask >> j) & 1)) ? member_ptr(a.w[j], bt.ws, mk) : nullptr;
    const double *V = member_ptr(a.V, bt.ws, mk);
    // 16-byte pairs (n4 is even, vectors start 16-byte aligned); the basis
    // is read four vectors at a time so that four independent loads are in
    // flight per thread, and each element still sums its terms in order
    const int n2 = n4 / 2;
    const size_t s2 = (size_t)n4 / 2;   // one basis vector, in pairs
    const double2 *V2 = reinterpret_cast<const double2 *>(V);
    double2 *y2 = reinterpret_cast<double2 *>(y);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += gridDim.x * blockDim.x) {
        double ax = 0.0, ay = 0.0;
        for (int j = 0; j < a.p; ++j)
            if (w[j]) {
                const double2 v = reinterpret_cast<const double2 *>(w[j])[i];
                ax += cf[j] * v.x;
                ay += cf[j] * v.y;
            }
        const double2 *vb = V2 + i;
        int k = 0;
        for (; k + 4 <= nb; k += 4) {
            const double2 v0 = vb[(size_t)k * s2], v1 = vb[(size_t)(k + 1) * s2];
            const double2 v2 = vb[(size_t)(k + 2) * s2], v3 = vb[(size_t)(k + 3) * s2];
            const double c0 = cf[a.p + k], c1 = cf[a.p + k + 1], c2 = cf[a.p + k + 2], c3 = cf[a.p + k + 3];
            ax += c0 * v0.x;
            ay += c0 * v0.y;
            ax += c1 * v1.x;
            ay += c1 * v1.y;
            ax += c2 * v2.x;
            ay += c2 * v2.y;
            ax += c3 * v3.x;
            ay += c3 * v3.y;
        }
        for (; k < nb; ++k) {
            const double2 v = vb[(size_t)k * s2];
            ax += cf[a.p + k] * v.x;
            ay += cf[a.p + k] * v.y;
        }
        y2[i] = make_double2(ax, ay);
    }
}

struct NormArgs {
    int nv;
    const double *vec[kPmax + 1];
};

__global__ void __launch_bounds__(kRedBlock) k_norms(int n4, NormArgs a, double *parts, Batch bt) {
    __shared__ double lds[16 * (kPmax + 1)];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const double *v[kPmax + 1];
    double r[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) {
        r[k] = 0.0;
        v[k] = (k < a.nv) ? member_ptr(a.vec[k], bt.ws, mk) : nullptr;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k <= kPmax; ++k) {
            if (k < a.nv) {
                const double x = v[k][i];
                r[k] += x * x;
            }
        }
    }
    block_sum_all<kPmax + 1>(r, lds);
    double *pk = parts + (size_t)mk * kVPartStride;
    if (threadIdx.x == 0)
        for (int k = 0; k < a.nv; ++k) pk[blockIdx.x * a.nv + k] = r[k];
}

struct CopyArgs {
    double *slot[8];
};

__global__ void __launch_bounds__(kBlock) k_copy_out(int n4, const double *__restrict__ y,
                                                     CopyArgs a, Batch bt) {
    const int mk = blockIdx.y;
    const int which = bt.pred.plan ? bt.pred.plan[kPlanW * mk + PF_COPY] - 1 : 0;
    if (which < 0 || which >= 8) return;
    y = member_ptr(y, bt.ws, mk);
    double *o = member_ptr(a.slot[which], bt.ws, mk);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x)
        o[i] = y[i];
}

__global__ void __launch_bounds__(kBlock) k_phi_init(PhiCtl *ctl0, int m0, const int32_t *m0k,
                                                     double tau0, double tol_rel,
                                                     const double *parts, int np, int nv,
                                                     double *vn2, Batch bt) {
    __shared__ double lds[16 * (kPmax + 1)];
    const int mk = blockIdx.x;
    if (!member_active(bt.pred, mk)) return;
    PhiCtl *c = ctl0 + mk;
    const double *pk = parts + (size_t)mk * kVPartStride;
    double tot[kPmax + 1];
#pragma unroll
    for (int k = 0; k <= kPmax; ++k) tot[k] = 0.0;
    for (int b = threadIdx.x; b < np; b += blockDim.x)
        for (int k = 0; k < nv; ++k) tot[k] += pk[b * nv + k];
    block_sum_all<kPmax + 1>(tot, lds);
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nv; ++k) {
        vn2[mk * (kPmax + 1) + k] = tot[k];
        const double r = sqrt(tot[k]);
        s = r > s ? r : s;
    }
    const int m = m0k ? m0k[mk] : m0;
    c->tol_abs = tol_rel * s;
    c->t = 0.0;
    c->tau = tau0;
    c->m = m;
    c->q = (m / 4.0 > 1.0) ? m / 4.0 : 1.0;
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
    c->dec.m_eff = 0;
}

// Layout change between the caller's component-major vectors
// [u_x | u_y | u_z | h] and the cell-major [cell][4] of the kernels, whose
// cell p is the caller's cell perm[p]; member k at src + k ss and dst + k ds.
// Element e of the cell-major side is component e & 3 of cell e >> 2, so
// that side is accessed contiguously (the other follows the cell order,
// whose chunks are compact patches).
template <bool TO_CELL>
__global__ void __launch_bounds__(kBlock) k_relayout(int n, const int32_t *__restrict__ perm,
                                                     const double *__restrict__ src, int64_t ss,
                                                     double *__restrict__ dst, int64_t ds) {
    const int mk = blockIdx.y;
    src += ss * mk;
    dst += ds * mk;
    const int n4 = 4 * n;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += gridDim.x * blockDim.x) {
        const size_t c = (size_t)(e & 3) * n + perm[e >> 2];
        if (TO_CELL)
            dst[e] = src[c];
        else
            dst[c] = src[e];
    }
}

}  // namespace

void launch_relayout(int n, const int32_t *perm, int nm, const double *src, int64_t ss, double *dst,
                     int64_t ds, bool to_cell, hipStream_t s) {
    const dim3 grid(grid_elems(4 * n), nm);
    if (to_cell)
        hipLaunchKernelGGL(k_relayout<true>, grid, dim3(kBlock), 0, s, n, perm, src, ss, dst, ds);
    else
        hipLaunchKernelGGL(k_relayout<false>, grid, dim3(kBlock), 0, s, n, perm, src, ss, dst, ds);
}

void launch_lincomb(int n4, double *out, int k, const double *const *vec, const double *c,
                    unsigned dtmask, const Batch &b, hipStream_t s) {
    LinArgs a{};
    a.k = k;
    a.dtmask = dtmask;
    for (int i = 0; i < k && i < kMaxLin; ++i) {
        a.vec[i] = vec[i];
        a.c[i] = c[i];
    }
    hipLaunchKernelGGL(k_lincomb, dim3(grid_elems(n4), b.nm), dim3(kBlock), 0, s, n4, out, a, b);
}

int launch_lincomb_dev(int n, double *out, int k, const double *const *vec,
                       const double *const *coef, PhiCtl *ctl0, double *nrm_out, const Batch &b,
                       hipStream_t s) {
    (void)ctl0;
    LinDevArgs a{};
    a.k = k;
    for (int i = 0; i < k && i <= kPmax; ++i) {
        a.vec[i] = vec[i];
        a.coef[i] = coef[i];
    }
    const int n4 = 4 * n;
    const int grid = red_parts(n);
    if (nrm_out)
        hipLaunchKernelGGL(k_lincomb_dev<true>, dim3(grid, b.nm), dim3(kRedBlock), 0, s, n4, out,
                           a, nrm_out, b);
    else
        hipLaunchKernelGGL(k_lincomb_dev<false>, dim3(grid, b.nm), dim3(kRedBlock), 0, s, n4, out,
                           a, nrm_out, b);
    return grid;
}

int launch_iom2_update(int n, int j, double *rjp1, const double *rj, const double *rjm1,
                       PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                       int np_dot, double *nrm_out, const Batch &b, hipStream_t s) {
    const int n4 = 4 * n;
    const int grid = upd_parts(n);
    hipLaunchKernelGGL(k_iom2_update, dim3(grid, b.nm), dim3(kRedBlock), 0, s, n4, j, rjp1, rj,
                       rjm1, ctl, nrm_in, np_nrm, dot_in, np_dot, nrm_out, b);
    return grid;
}

void launch_combine(int n4, double *y, int p, const double *const *w, const int *wzero,
                    const double *V, PhiCtl *ctl, const Batch &b, hipStream_t s) {
    CombArgs a{};
    a.p = p;
    for (int j = 0; j < p; ++j) a.w[j] = wzero[j] ? nullptr : w[j];
    a.V = V;
    hipLaunchKernelGGL(k_combine, dim3(grid_elems(n4 / 2), b.nm), dim3(kBlock), 0, s, n4, y, a, ctl, b);
}

int launch_norms(int n, int nv, const double *const *vec, double *parts, const Batch &b,
                 hipStream_t s) {
    NormArgs a{};
    a.nv = nv;
    for (int k = 0; k < nv && k <= kPmax; ++k) a.vec[k] = vec[k];
    const int grid = red_parts(n);
    hipLaunchKernelGGL(k_norms, dim3(grid, b.nm), dim3(kRedBlock), 0, s, 4 * n, a, parts, b);
    return grid;
}

void launch_copy_out(int n4, const double *y, double *const *slots, const Batch &b,
                     hipStream_t s) {
    CopyArgs a{};
    for (int k = 0; k < 8; ++k) a.slot[k] = slots[k];
    hipLaunchKernelGGL(k_copy_out, dim3(grid_elems(n4), b.nm), dim3(kBlock), 0, s, n4, y, a, b);
}

void launch_phi_init(PhiCtl *ctl, int m0, const int32_t *m0k, double tau0, double tol_rel,
                     const double *parts, int np, int nv, double *vnorm2, const Batch &b,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_phi_init, dim3(b.nm), dim3(kBlock), 0, s, ctl, m0, m0k, tau0, tol_rel,
                       parts, np, nv, vnorm2, b);
}

}  // namespace xrb
