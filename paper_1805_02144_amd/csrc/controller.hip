// Per-attempt kernel of phipm_simul_iom2 (Alg. 1, steps 2(ii)-6), one
// 256-thread workgroup:
//   * X = exp(tau Hhat) of the augmented IOM2 Hessenberg matrix
//     Hhat = [[H_m, e_1 e_1^T], [0, N_{p+1}]] (remark after Alg. 1), by a
//     degree-13 Pade approximant with scaling and squaring -- the method whose
//     flop count (44/3 + 2 s) K^3 eq. cost prices;
//   * error estimate eps = beta h_{m+1,m} |X(m, m+p+1)| and
//     omega = t_out eps / (tau Tol) (steps 3 and 6);
//   * (tau, m) update with the cost comparison of eq. cost (steps 4-5);
//   * on acceptance, the coefficients of y_{k+1} (eq. 3.17) for the
//     combination kernel and t^l/l! for the next w_j recurrence (eq. 3.18).
// Matrices live in LDS (K <= 49, padded to 52); products use one 4x4
// register tile per thread.
#include "column.h"
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

constexpr int kLd = 52;                 // padded order, multiple of 4, >= kKmax
constexpr int kMat = kLd * kLd;
static_assert(kLd >= kKmax && kLd % 4 == 0, "LDS matrix padding");

// C = A B over the leading K4 x K4 block (K4 multiple of 4).  Register tiles
// of T x T per thread: T = 2 while (K4/2)^2 threads fit the block, else 4.
template <int T>
__device__ inline void mat_mul_tiles(const double *A, const double *B, double *C, int K4) {
    const int nt = K4 / T;
    for (int tile = threadIdx.x; tile < nt * nt; tile += blockDim.x) {
        const int r0 = (tile / nt) * T, c0 = (tile % nt) * T;
        double acc[T][T];
#pragma unroll
        for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) acc[r][c] = 0.0;
        for (int k = 0; k < K4; ++k) {
            double a[T], b[T];
#pragma unroll
            for (int r = 0; r < T; ++r) a[r] = A[(r0 + r) * kLd + k];
#pragma unroll
            for (int c = 0; c < T; ++c) b[c] = B[k * kLd + c0 + c];
#pragma unroll
            for (int r = 0; r < T; ++r)
#pragma unroll
                for (int c = 0; c < T; ++c) acc[r][c] += a[r] * b[c];
        }
#pragma unroll
        for (int r = 0; r < T; ++r)
#pragma unroll
            for (int c = 0; c < T; ++c) C[(r0 + r) * kLd + c0 + c] = acc[r][c];
    }
}

__device__ void mat_mul(const double *A, const double *B, double *C, int K4) {
    if ((K4 / 2) * (K4 / 2) <= (int)blockDim.x) mat_mul_tiles<2>(A, B, C, K4);
    else mat_mul_tiles<4>(A, B, C, K4);
    __syncthreads();
}

// round x > 0 down to two significant digits with exact decimal scalings
__device__ double quantise_2sig(double x) {
#pragma clang fp contract(off)
    if (!(x > 0.0) || !(x < 1e300)) return x;
    double p = 1.0;
    for (int it = 0; it < 400 && p > x; ++it) p = p / 10.0;
    for (int it = 0; it < 400 && p * 10.0 <= x; ++it) p = p * 10.0;
    const double unit = p / 10.0;
    return floor(x / unit) * unit;
}

// eq. cost with n_A = 40 n
__device__ double work_estimate(double tau, int m, int p, double t, double t_out, double n,
                                double normH, double tau_ref) {
#pragma clang fp contract(off)
    const double nA = 40.0 * n;
    double steps = round((t_out - t) / tau);
    if (steps < 1.0) steps = 1.0;
    double M = 44.0 / 3.0;
    const double hn = normH * tau / tau_ref;
    if (hn > 0.0) {
        const double r = round(log2(hn / 5.37));
        if (r > 0.0) M = M + 2.0 * r;
    }
    const double K = (double)(m + p + 1);
    return steps * m * (n + nA) + 2.0 * (p - 1) * (nA + n) + M * K * K * K + (2.0 * p + 1.0) * n;
}

__global__ void __launch_bounds__(kBlock) k_controller(PhiCtl *ctl0, CtlArgs a0,
                                                       const CtlArgs *dargs, double *nrm_parts,
                                                       Batch bt) {
    const int mk = blockIdx.x;
    if (!member_active(bt.pred, mk)) return;
    PhiCtl *c = ctl0 + mk;
    const CtlArgs a = dargs ? dargs[mk] : a0;
    const double *nrm_in = nrm_parts + (size_t)mk * kPartStride + (size_t)a.nrm_buf * kRedBlocks;
    __shared__ double Bm[kMat], B2[kMat], B4[kMat], B6[kMat], Um[kMat], Vm[kMat];
    __shared__ double mult[kLd];
    __shared__ double sh_tau_u, sh_norm, sh_hsub;
    __shared__ int sh_lands, sh_meff, sh_s, sh_piv, sh_status;
    __shared__ double red[32];
    const int tid = threadIdx.x;
    const int p = a.p;
    const int m = a.m;

    // finish the norm of the last IOM2 column (h_{built,built-1} or beta)
    if (!a.wp_zero && a.built >= 1) {
        const bool live = (c->brk == 0) && !c->beta_zero;
        if (live) {
            double tot[1];
            sum_partials<1>(tot, nrm_in, a.n_nrm_in, red);
            finalize_column(c, a.built, tot[0], tid == 0, red);
        }
        __syncthreads();
    }

    if (tid == 0) {
#pragma clang fp contract(off)
        c->t_out = a.t_out;
        double tau_u;
        int lands;
        if (a.mode == XRB_REPLAY) {
            tau_u = a.rep.tau;
            lands = (a.rep.flags >> 1) & 1;
        } else {
            const double rem = a.t_out - c->t;
            if (c->tau >= rem * (1.0 - 1e-12)) {
                tau_u = rem;
                lands = 1;
            } else {
                tau_u = c->tau;
                lands = 0;
            }
        }
        sh_tau_u = tau_u;
        sh_lands = lands;
        int status = c->dec.status;
        if (c->beta != c->beta) status = XRB_ENAN;
        sh_status = status;
        const int beta_zero = a.wp_zero || c->beta_zero;
        int meff = 0;
        double hsub = 0.0;
        if (!beta_zero) {
            const int brk = c->brk;
            meff = (brk > 0 && brk < m) ? brk : m;
            hsub = (brk > 0 && meff == brk) ? 0.0 : c->H[meff * kMmax + meff - 1];
        }
        sh_meff = beta_zero ? 0 : meff;
        sh_hsub = hsub;
    }
    __syncthreads();
    const int meff = sh_meff;
    const double tau_u = sh_tau_u;
    int K = 0, K4 = 0;
    double *X = nullptr;

    if (meff > 0) {
        K = meff + p + 1;
        K4 = (K + 3) & ~3;
        // Hhat scaled by tau_u, zero padded
        for (int e = tid; e < kLd * kLd; e += blockDim.x) {
            const int r = e / kLd, q = e % kLd;
            double v = 0.0;
            if (r < meff && q < meff) v = tau_u * c->H[r * kMmax + q];
            else if (r == 0 && q == meff) v = tau_u;
            else if (r >= meff && r < meff + p && q == r + 1) v = tau_u;
            Bm[e] = v;
        }
        __syncthreads();
        // 1-norm of tau Hhat: a column per thread
        double csum = 0.0;
        if (tid < K)
            for (int r = 0; r < K; ++r) csum += fabs(Bm[r * kLd + tid]);
        const double nrm = block_max(csum, red);
        if (tid == 0) {
            int s = 0;
            double sc = 1.0;
            if (!(nrm < 1e300)) {
                sh_status = XRB_ENAN;   // non-finite Hessenberg entries
            } else {
                while (nrm * sc > 5.371920351148152) {
                    ++s;
                    sc *= 0.5;
                }
            }
            sh_norm = nrm;
            sh_s = s;
            mult[0] = sc;
        }
        __syncthreads();
        const double sc = mult[0];
        for (int e = tid; e < kMat; e += blockDim.x) Bm[e] *= sc;
        __syncthreads();
        // Pade [13/13] numerator coefficients from the closed form, b_0 = 1
        double b[14];
        b[0] = 1.0;
        for (int j = 0; j < 13; ++j) b[j + 1] = b[j] * (13.0 - j) / ((26.0 - j) * (j + 1.0));
        mat_mul(Bm, Bm, B2, K4);
        mat_mul(B2, B2, B4, K4);
        mat_mul(B4, B2, B6, K4);
        // even part V = B6 (b12 B6 + b10 B4 + b8 B2) + b6 B6 + b4 B4 + b2 B2 + b0 I
        for (int e = tid; e < kMat; e += blockDim.x) Um[e] = b[12] * B6[e] + b[10] * B4[e] + b[8] * B2[e];
        __syncthreads();
        mat_mul(B6, Um, Vm, K4);
        for (int e = tid; e < kMat; e += blockDim.x) {
            const int r = e / kLd, q = e % kLd;
            Vm[e] += b[6] * B6[e] + b[4] * B4[e] + b[2] * B2[e] + ((r == q && r < K) ? b[0] : 0.0);
        }
        // odd part U = B (B6 (b13 B6 + b11 B4 + b9 B2) + b7 B6 + b5 B4 + b3 B2 + b1 I)
        for (int e = tid; e < kMat; e += blockDim.x) Um[e] = b[13] * B6[e] + b[11] * B4[e] + b[9] * B2[e];
        __syncthreads();
        for (int e = tid; e < kMat; e += blockDim.x) {
            const int r = e / kLd, q = e % kLd;
            B2[e] = b[7] * B6[e] + b[5] * B4[e] + b[3] * B2[e] + ((r == q && r < K) ? b[1] : 0.0);
        }
        __syncthreads();
        mat_mul(B6, Um, B4, K4);
        for (int e = tid; e < kMat; e += blockDim.x) B4[e] += B2[e];
        __syncthreads();
        mat_mul(Bm, B4, B6, K4);              // B6 <- U
        // (V - U) X = (V + U): M in B4, right-hand sides in Vm
        for (int e = tid; e < kMat; e += blockDim.x) {
            const double v = Vm[e], u = B6[e];
            B4[e] = v - u;
            Vm[e] = v + u;
        }
        __syncthreads();
        double *Mt = B4, *R = Vm;
        for (int col = 0; col < K; ++col) {
            // partial pivoting: first row of largest |M(r, col)|, one wave
            if (tid < 64) {
                double best = -1.0;
                int piv = K;
                for (int r = col + tid; r < K; r += 64) {
                    const double v = fabs(Mt[r * kLd + col]);
                    if (v > best) {
                        best = v;
                        piv = r;
                    }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_down(best, off, 64);
                    const int op = __shfl_down(piv, off, 64);
                    if (ob > best || (ob == best && op < piv)) {
                        best = ob;
                        piv = op;
                    }
                }
                if (tid == 0) {
                    sh_piv = piv;
                    if (!(best > 0.0)) sh_status = XRB_ENAN;
                }
            }
            __syncthreads();
            const int piv = sh_piv < K ? sh_piv : col;
            if (piv != col) {
                for (int q = tid; q < K; q += blockDim.x) {
                    double t = Mt[col * kLd + q];
                    Mt[col * kLd + q] = Mt[piv * kLd + q];
                    Mt[piv * kLd + q] = t;
                    t = R[col * kLd + q];
                    R[col * kLd + q] = R[piv * kLd + q];
                    R[piv * kLd + q] = t;
                }
                __syncthreads();
            }
            const double dinv = 1.0 / Mt[col * kLd + col];
            const int rows = K - col - 1;
            // rank-1 update of the trailing rows of M (columns > col) and R
            const int width = (K - col - 1) + K;
            for (int e = tid; e < rows * width; e += blockDim.x) {
                const int r = col + 1 + e / width, q = e % width;
                const double l = Mt[r * kLd + col] * dinv;
                if (q < K - col - 1) {
                    const int qq = col + 1 + q;
                    Mt[r * kLd + qq] -= l * Mt[col * kLd + qq];
                } else {
                    const int qq = q - (K - col - 1);
                    R[r * kLd + qq] -= l * R[col * kLd + qq];
                }
            }
            __syncthreads();
        }
        // back substitution, column-oriented: X(r,:) = R(r,:)/M(r,r), then
        // R(i,:) -= M(i,r) X(r,:) for i < r
        for (int r = K - 1; r >= 0; --r) {
            const double dinv = 1.0 / Mt[r * kLd + r];
            for (int q = tid; q < K; q += blockDim.x) R[r * kLd + q] *= dinv;
            __syncthreads();
            for (int e = tid; e < r * K; e += blockDim.x) {
                const int i = e / K, q = e % K;
                R[i * kLd + q] -= Mt[i * kLd + r] * R[r * kLd + q];
            }
            __syncthreads();
        }
        // zero the padding of R before squaring
        for (int e = tid; e < kMat; e += blockDim.x) {
            const int r = e / kLd, q = e % kLd;
            if (r >= K || q >= K) R[e] = 0.0;
        }
        __syncthreads();
        X = R;
        double *T = B4;
        for (int q = 0; q < sh_s; ++q) {
            mat_mul(X, X, T, K4);
            double *tmp = X;
            X = T;
            T = tmp;
        }
        __syncthreads();
    }

    if (tid == 0) {
#pragma clang fp contract(off)
        int status = sh_status;
        int accept;
        double omega = 0.0;
        const double beta = c->beta;
        if (meff == 0) {
            accept = 1;   // w_p = 0: the substep is exact
        } else {
            const double eps = beta * sh_hsub * fabs(X[(meff - 1) * kLd + meff + p]);
            omega = c->t_out * eps / (tau_u * c->tol_abs);
            if (omega != omega) status = XRB_ENAN;
            accept = (a.mode == XRB_REPLAY) ? (a.rep.flags & 1) : (omega <= a.delta);
        }
        int m_next = m;
        if (a.mode != XRB_REPLAY && meff > 0) {
            // order / error-ratio estimates from the previous rejected attempt
            if (c->have_prev && omega > 0.0 && c->prev_omega > 0.0) {
                if (m == c->prev_m && tau_u != c->prev_tau) {
                    const double qq = log(omega / c->prev_omega) / log(tau_u / c->prev_tau);
                    c->q = qq > 1.0 ? qq : 1.0;
                } else if (tau_u == c->prev_tau && m != c->prev_m) {
                    const double kk = pow(omega / c->prev_omega, 1.0 / (double)(c->prev_m - m));
                    c->kappa = kk > 1.1 ? kk : 1.1;
                }
            }
            double tau_new, mnew;
            if (omega > 0.0) {
                tau_new = tau_u * pow(a.gamma / omega, 1.0 / c->q);
                mnew = (double)m + ceil(log(omega / a.gamma) / log(c->kappa));
            } else {
                tau_new = 2.0 * tau_u;
                mnew = -1e300;
            }
            if (tau_new > 2.0 * tau_u) tau_new = 2.0 * tau_u;
            if (tau_new < tau_u / 5.0) tau_new = tau_u / 5.0;
            tau_new = quantise_2sig(tau_new);
            int lo = (3 * m + 3) / 4;
            if (lo < 1) lo = 1;
            int hi = (4 * m) / 3 + 1;
            if (hi > a.m_max) hi = a.m_max;
            if (mnew < lo) mnew = lo;
            if (mnew > hi) mnew = hi;
            const int m_new = (int)mnew;
            const double c_tau = work_estimate(tau_new, m, p, c->t, c->t_out, a.n4, sh_norm, tau_u);
            const double c_m = work_estimate(tau_u, m_new, p, c->t, c->t_out, a.n4, sh_norm, tau_u);
            int change_tau = c_tau < c_m;
            if (!accept && !change_tau && m_new == m) change_tau = 1;
            if (change_tau) c->tau = tau_new;
            else m_next = m_new;
        }
        c->m = m_next;
        // combine coefficients: tau^j/j! w_j, beta sigma_k X(k, m+p-1), correction
        double fac = 1.0;
        for (int j = 0; j < p; ++j) {
            if (j > 0) fac = fac * tau_u / j;
            c->ycoef[j] = fac;
        }
        if (meff > 0) {
            const int cmain = p > 0 ? meff + p - 1 : 0;
            for (int k = 0; k < meff; ++k) c->ycoef[p + k] = beta * c->sigma[k] * X[k * kLd + cmain];
            c->ycoef[p + meff] = beta * sh_hsub * c->sigma[meff] * X[(meff - 1) * kLd + meff + p];
        }
        double t_new = c->t;
        if (accept) {
            t_new = sh_lands ? c->t_out : c->t + tau_u;
            c->t = t_new;
            c->have_prev = 0;
            double f2 = 1.0;
            c->rec_coef[0] = 1.0;
            for (int l = 1; l <= kPmax; ++l) {
                f2 = f2 * t_new / l;
                c->rec_coef[l] = f2;
            }
        } else {
            c->have_prev = 1;
            c->prev_omega = omega;
            c->prev_tau = tau_u;
            c->prev_m = m;
        }
        c->dec.tau_u = tau_u;
        c->dec.omega = omega;
        c->dec.t = t_new;
        c->dec.accept = accept;
        c->dec.lands = sh_lands;
        c->dec.m_next = m_next;
        c->dec.m_eff = meff;
        c->dec.status = status;
        c->dec.reached = (t_new >= c->t_out) ? 1 : 0;
    }
}

}  // namespace

void launch_controller(PhiCtl *ctl, const CtlArgs &a, const CtlArgs *dargs, double *nrm_parts,
                       const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_controller, dim3(b.nm), dim3(kBlock), 0, s, ctl, a, dargs, nrm_parts, b);
}

}  // namespace xrb
