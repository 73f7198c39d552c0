// Per-attempt kernel of phipm_simul_iom2 (Alg. 1, steps 2(ii)-6), one
// 256-thread workgroup:
//   * X = exp(tau Hhat) of the augmented IOM2 Hessenberg matrix
//     Hhat = [[H_m, e_1 e_1^T], [0, N_{p+1}]] (remark after Alg. 1), by the
//     degree-16 Taylor polynomial in Paterson-Stockmeyer form with scaling
//     and squaring: products only, every one on the FP64 matrix cores (a
//     Pade approximant would need a pivoted solve, whose one barrier per
//     column cost more here than the whole polynomial);
//   * error estimate eps = beta h_{m+1,m} |X(m, m+p+1)| and
//     omega = t_out eps / (tau Tol) (steps 3 and 6);
//   * (tau, m) update with the cost comparison of eq. cost (steps 4-5; the
//     cost model prices the exponential as the paper does, by the degree-13
//     Pade flop count (44/3 + 2 s) K^3);
//   * on acceptance, the coefficients of y_{k+1} (eq. 3.17) for the
//     combination kernel and t^l/l! for the next w_j recurrence (eq. 3.18).
// Matrices live in LDS (K <= 49, padded to 52).  The matrix products run on
// the FP64 matrix cores (16 x 16 tiles, one wave per tile).
#include "column.h"
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

constexpr int kLd = 52;                 // padded order, multiple of 4, >= kKmax
constexpr int kMat = kLd * kLd;
static_assert(kLd >= kKmax && kLd % 4 == 0, "LDS matrix padding");

typedef double dbl4 __attribute__((ext_vector_type(4)));

// The dense part works on size classes KC in {16, 32, 52} (KC >= K4, rows
// and columns below KC <= kLd are inside the LDS matrices), so that loops
// unroll to fixed trip counts.  Loads are unconditional at in-range
// addresses and masked by a select, with no branch between them: the LDS
// reads of a phase then go out back to back.

// Products on the FP64 matrix cores.  C = A B over the leading K4 x K4
// block (K4 a multiple of 4), cut into 16 x 16 output tiles, one wave per
// tile at a time; each tile is K4/4 rank-4 steps of v_mfma_f64_16x16x4.
// Lane l supplies A(i0 + l%16, k0 + l/16) and B(k0 + l/16, j0 + l%16) and
// holds C(i0 + l/16 + 4 v, j0 + l%16), v < 4.  Entries at or past K4 enter
// as zeros and are never written.  The accumulator starts from
// init(nb, row, col) (a term added to the product) and each result goes to
// store(e, values), e the entry's LDS index, so elementwise terms fuse into
// the product pass.
// NB operand pairs share one pass (the same A, NB right-hand factors).
template <int KC, int NB, class Init, class Store>
__device__ inline void mfma_pass(const double *A, const double *const (&B)[NB], int K4, Init init,
                                 Store store) {
    constexpr int KS = KC / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = (K4 + 15) >> 4;
    const int li = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < nt * nt; tile += (int)(blockDim.x >> 6)) {
        const int i0 = (tile / nt) << 4, j0 = (tile % nt) << 4;
        const int col = j0 + li, ar = i0 + li;
        const int colc = col < kLd ? col : kLd - 1, arc = ar < kLd ? ar : kLd - 1;
        double af[KS], bf[NB][KS];
#pragma unroll
        for (int st = 0; st < KS; ++st) {
            const int k = 4 * st + lk;
            const bool ks = 4 * st < K4;
            const double av = A[arc * kLd + k];
            af[st] = (ks && ar < K4) ? av : 0.0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const double bv = B[nb][k * kLd + colc];
                bf[nb][st] = (ks && col < K4) ? bv : 0.0;
            }
        }
        dbl4 acc[NB];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = i0 + lk + 4 * v;
            const int rowc = row < kLd ? row : kLd - 1;
            const bool in = row < K4 && col < K4;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const double iv = init(nb, rowc, colc);
                acc[nb][v] = in ? iv : 0.0;
            }
        }
#pragma unroll
        for (int st = 0; st < KS; ++st)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[st], bf[nb][st], acc[nb], 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = i0 + lk + 4 * v;
            if (row < K4 && col < K4) {
                double out[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) out[nb] = acc[nb][v];
                store(row * kLd + col, out);
            }
        }
    }
    __syncthreads();
}

template <int KC>
__device__ inline void mat_mul(const double *A, const double *B, double *C, int K4) {
    const double *const bb[1] = {B};
    mfma_pass<KC, 1>(A, bb, K4, [](int, int, int) { return 0.0; },
                     [C](int e, const double(&v)[1]) { C[e] = v[0]; });
}

// lane l's v, the same in every lane
__device__ inline double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Taylor coefficients 1/k!, k = 0..16 (evaluated at compile time with the
// same IEEE operations as at run time)
struct Taylor16 {
    double c[17];
};
constexpr Taylor16 taylor16() {
    Taylor16 t{};
    t.c[0] = 1.0;
    for (int k = 1; k <= 16; ++k) t.c[k] = t.c[k - 1] / k;
    return t;
}
// The scaled matrix's 1-norm bound: for ||B||_1 <= 0.75 the remainder of the
// degree-16 series, sum_{k>16} B^k/k!, is below 0.75^17/17! e^0.75 / (1 - 0.75/18)
// < 5e-17 in norm against ||e^B|| >= e^-0.75, under half a unit roundoff
// relative to the result.
constexpr double kTaylorTheta = 0.75;

// LDS matrices of the exponential (each kLd x kLd)
struct ExpmLds {
    double *B1, *B2, *B3, *B4, *T, *U;
};

// exp(B1)^(2^n_sq) for the scaled matrix B1 of order K (zero padded), the
// polynomial as sum_i B^4i A_i with A_i = c_4i I + c_4i+1 B + c_4i+2 B^2 +
// c_4i+3 B^3 (i < 4) plus c_16 B^16, by Horner in B^4: B^2, then B^3 and B^4
// in one pass (the innermost block A_3 + c_16 B^4 formed in its epilogue),
// three Horner products with A_i added in their epilogues, then the
// squarings.  The result is one of the LDS matrices, returned.
template <int KC>
__device__ double *taylor16_expm(const ExpmLds &L, int K, int K4, int n_sq) {
    constexpr Taylor16 kTay = taylor16();
    const double *c = kTay.c;
    double *B1 = L.B1, *B2 = L.B2, *B3 = L.B3, *B4 = L.B4;
    mat_mul<KC>(B1, B1, B2, K4);
    {
        const double *const bb[2] = {B1, B2};
        double *T = L.T;
        mfma_pass<KC, 2>(B2, bb, K4, [](int, int, int) { return 0.0; },
                         [&](int e, const double(&v)[2]) {
                             B3[e] = v[0];
                             B4[e] = v[1];
                             const int r = e / kLd, col = e - r * kLd;
                             const double id = (r == col && r < K) ? 1.0 : 0.0;
                             T[e] = c[12] * id + c[13] * B1[e] + c[14] * B2[e] + c[15] * v[0] + c[16] * v[1];
                         });
    }
    double *src = L.T, *dst = L.U;
    for (int i = 2; i >= 0; --i) {
        const double *const bb[1] = {src};
        mfma_pass<KC, 1>(B4, bb, K4,
                         [&](int, int r, int col) {
                             const int e = r * kLd + col;
                             const double id = (r == col && r < K) ? 1.0 : 0.0;
                             return c[4 * i] * id + c[4 * i + 1] * B1[e] + c[4 * i + 2] * B2[e] +
                                    c[4 * i + 3] * B3[e];
                         },
                         [&](int e, const double(&v)[1]) { dst[e] = v[0]; });
        double *tmp = src;
        src = dst;
        dst = tmp;
    }
    double *X = src, *Y = dst;
    for (int q = 0; q < n_sq; ++q) {
        mat_mul<KC>(X, X, Y, K4);
        double *tmp = X;
        X = Y;
        Y = tmp;
    }
    return X;
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
                                                       Decision *hdec, int seq, Batch bt) {
    const int mk = blockIdx.x;
    if (!member_active(bt.pred, mk)) return;
    PhiCtl *c = ctl0 + mk;
    const CtlArgs a = dargs ? dargs[mk] : a0;
    const double *nrm_in = nrm_parts + (size_t)mk * kPartStride + (size_t)a.nrm_buf * kNrmRegion;
    __shared__ double Bm[kMat], B2[kMat], B3[kMat], B4[kMat], Tm[kMat], Um[kMat];
    __shared__ double sh_tau_u, sh_norm, sh_hsub;
    __shared__ int sh_lands, sh_meff, sh_status;
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
    int K = 0, K4 = 0, n_sq = 0;
    double *X = nullptr;

    if (meff > 0) {
        K = meff + p + 1;
        K4 = (K + 3) & ~3;
        // 2^-s tau Hhat.  Thread q < m reads the IOM2 band of column q of H
        // (rows q-1, q, q+1; H is zero elsewhere) and the threads of the
        // augmentation columns hold their single tau; the 1-norm is the
        // largest column sum.  Every thread derives s from it alike.
        double hv0 = 0.0, hv1 = 0.0, hv2 = 0.0, csum = 0.0;
        if (tid < meff) {
            if (tid > 0) hv0 = tau_u * c->H[(tid - 1) * kMmax + tid];
            hv1 = tau_u * c->H[tid * kMmax + tid];
            if (tid + 1 < meff) hv2 = tau_u * c->H[(tid + 1) * kMmax + tid];
            csum = fabs(hv0) + fabs(hv1) + fabs(hv2);
        } else if (tid < K) {
            csum = fabs(tau_u);
        }
        for (int e = tid; e < kMat; e += blockDim.x) Bm[e] = 0.0;
        const double nrm = block_max(csum, red);
        double sc = 1.0;
        if (!(nrm < 1e300)) {
            if (tid == 0) sh_status = XRB_ENAN;   // non-finite Hessenberg entries
        } else {
            while (nrm * sc > kTaylorTheta) {
                ++n_sq;
                sc *= 0.5;
            }
        }
        if (tid == 0) sh_norm = nrm;
        if (tid < meff) {
            if (tid > 0) Bm[(tid - 1) * kLd + tid] = hv0 * sc;
            Bm[tid * kLd + tid] = hv1 * sc;
            if (tid + 1 < meff) Bm[(tid + 1) * kLd + tid] = hv2 * sc;
        } else if (tid == meff) {
            Bm[meff] = tau_u * sc;                    // row 0 (e_1 e_1^T block)
        } else if (tid < K) {
            Bm[(tid - 1) * kLd + tid] = tau_u * sc;   // superdiagonal of N_{p+1}
        }
        __syncthreads();
        const ExpmLds L{Bm, B2, B3, B4, Tm, Um};
        if (K4 <= 16) X = taylor16_expm<16>(L, K, K4, n_sq);
        else if (K4 <= 32) X = taylor16_expm<32>(L, K, K4, n_sq);
        else X = taylor16_expm<kLd>(L, K, K4, n_sq);
    }

    // combination coefficients of the basis, beta sigma_k X(k, m+p-1), a row per thread
    if (meff > 0) {
        const int cmain = p > 0 ? meff + p - 1 : 0;
        const double beta = c->beta;
        for (int k = tid; k < meff; k += blockDim.x) c->ycoef[p + k] = beta * c->sigma[k] * X[k * kLd + cmain];
    }
    // The scalar controller (steps 3-6) runs on the first wave: every lane
    // evaluates omega and the history update alike, then lane 1 the new
    // substep (and its cost), lane 2 the new Krylov size (and its cost),
    // lanes 3 and 4 the combination and recurrence coefficients, side by side;
    // lane 0 takes the decision and writes the record.  Each quantity is the
    // same expression one thread evaluated before, so the bits are unchanged.
    if (tid < 64) {
#pragma clang fp contract(off)
        const int lane = tid;
        int status = sh_status;
        int accept;
        double omega = 0.0;
        const double beta = c->beta;
        const double t_cur = c->t, t_out = c->t_out;
        if (meff == 0) {
            accept = 1;   // w_p = 0: the substep is exact
        } else {
            const double eps = beta * sh_hsub * fabs(X[(meff - 1) * kLd + meff + p]);
            omega = t_out * eps / (tau_u * c->tol_abs);
            if (omega != omega) status = XRB_ENAN;
            accept = (a.mode == XRB_REPLAY) ? (a.rep.flags & 1) : (omega <= a.delta);
        }
        int m_next = m;
        if (a.mode != XRB_REPLAY && meff > 0) {
            // order / error-ratio estimates from the previous rejected attempt
            double q = c->q, kappa = c->kappa;
            if (c->have_prev && omega > 0.0 && c->prev_omega > 0.0) {
                if (m == c->prev_m && tau_u != c->prev_tau) {
                    const double qq = log(omega / c->prev_omega) / log(tau_u / c->prev_tau);
                    q = qq > 1.0 ? qq : 1.0;
                } else if (tau_u == c->prev_tau && m != c->prev_m) {
                    const double kk = pow(omega / c->prev_omega, 1.0 / (double)(c->prev_m - m));
                    kappa = kk > 1.1 ? kk : 1.1;
                }
            }
            double tau_new = 0.0, c_tau = 0.0, c_m = 0.0;
            int m_new = m;
            if (lane == 1) {
                if (omega > 0.0) tau_new = tau_u * pow(a.gamma / omega, 1.0 / q);
                else tau_new = 2.0 * tau_u;
                if (tau_new > 2.0 * tau_u) tau_new = 2.0 * tau_u;
                if (tau_new < tau_u / 5.0) tau_new = tau_u / 5.0;
                tau_new = quantise_2sig(tau_new);
                c_tau = work_estimate(tau_new, m, p, t_cur, t_out, a.n4, sh_norm, tau_u);
            } else if (lane == 2) {
                double mnew;
                if (omega > 0.0) mnew = (double)m + ceil(log(omega / a.gamma) / log(kappa));
                else mnew = -1e300;
                int lo = (3 * m + 3) / 4;
                if (lo < 1) lo = 1;
                int hi = (4 * m) / 3 + 1;
                if (hi > a.m_max) hi = a.m_max;
                if (mnew < lo) mnew = lo;
                if (mnew > hi) mnew = hi;
                m_new = (int)mnew;
                c_m = work_estimate(tau_u, m_new, p, t_cur, t_out, a.n4, sh_norm, tau_u);
            }
            tau_new = read_lane(tau_new, 1);
            c_tau = read_lane(c_tau, 1);
            m_new = __builtin_amdgcn_readlane(m_new, 2);
            c_m = read_lane(c_m, 2);
            int change_tau = c_tau < c_m;
            if (!accept && !change_tau && m_new == m) change_tau = 1;
            if (change_tau) {
                if (lane == 0) c->tau = tau_new;
            } else {
                m_next = m_new;
            }
            if (lane == 0) {
                c->q = q;
                c->kappa = kappa;
            }
        }
        if (lane == 0) c->m = m_next;
        // combine coefficients: tau^j/j! w_j, beta sigma_k X(k, m+p-1), correction
        if (lane == 3) {
            double fac = 1.0;
            for (int j = 0; j < p; ++j) {
                if (j > 0) fac = fac * tau_u / j;
                c->ycoef[j] = fac;
            }
            if (meff > 0)
                c->ycoef[p + meff] = beta * sh_hsub * c->sigma[meff] * X[(meff - 1) * kLd + meff + p];
        }
        const double t_new = accept ? (sh_lands ? t_out : t_cur + tau_u) : t_cur;
        if (accept) {
            if (lane == 4) {
                double f2 = 1.0;
                c->rec_coef[0] = 1.0;
                for (int l = 1; l <= kPmax; ++l) {
                    f2 = f2 * t_new / l;
                    c->rec_coef[l] = f2;
                }
            }
            if (lane == 0) {
                c->t = t_new;
                c->have_prev = 0;
            }
        } else if (lane == 0) {
            c->have_prev = 1;
            c->prev_omega = omega;
            c->prev_tau = tau_u;
            c->prev_m = m;
        }
        if (lane != 0) return;
        Decision d;
        d.tau_u = tau_u;
        d.omega = omega;
        d.t = t_new;
        d.accept = accept;
        d.lands = sh_lands;
        d.m_next = m_next;
        d.m_eff = meff;
        d.status = status;
        d.reached = (t_new >= c->t_out) ? 1 : 0;
        d.seq = 0;
        c->dec = d;
        // the host copy: record first, then its sequence number behind a
        // system-scope release (vector stores to mapped host memory)
        hdec[mk] = d;
        __hip_atomic_store(&hdec[mk].seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

void launch_controller(PhiCtl *ctl, const CtlArgs &a, const CtlArgs *dargs, double *nrm_parts,
                       Decision *hdec, int seq, const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_controller, dim3(b.nm), dim3(kBlock), 0, s, ctl, a, dargs, nrm_parts, hdec,
                       seq, b);
}

}  // namespace xrb
