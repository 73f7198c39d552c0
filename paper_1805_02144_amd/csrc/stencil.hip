// Finite-volume stencil kernels of the shallow-water model (Sec. 2):
//   F(u)    eq. sweqsinv with D_f = -nu L^2 (eq. swdis)
//   J(u) x  eqs. dynjs-dynjc, fused with the IOM2 dot products or the w_j
//           recurrence axpys of Alg. 1
// One thread per cell, neighbours gathered through the slot-major table.
// The two-ring dissipation stencil L(L x) takes L x from a preceding
// one-ring pass (launch_lap4).
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

inline int grid_for(int n) {
    int g = (n + kBlock - 1) / kBlock;
    return g < 1 ? 1 : g;
}
inline int grid_capped(int n) {
    int g = grid_for(n);
    return g > kMaxBlocks ? kMaxBlocks : g;
}

__global__ void __launch_bounds__(kBlock) k_lap4(DevMesh M, const double *__restrict__ psi,
                                                 double *__restrict__ out) {
    const int n = M.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p0 = psi[i], p1 = psi[n + i], p2 = psi[2 * n + i], p3 = psi[3 * n + i];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = M.nbr[s * n + i];
        const double c = M.cl[s * n + i];
        a0 += c * (psi[j] - p0);
        a1 += c * (psi[n + j] - p1);
        a2 += c * (psi[2 * n + j] - p2);
        a3 += c * (psi[3 * n + j] - p3);
    }
    out[i] = a0;
    out[n + i] = a1;
    out[2 * n + i] = a2;
    out[3 * n + i] = a3;
}

__global__ void __launch_bounds__(kBlock) k_linearize(DevMesh M, const double *__restrict__ u,
                                                      double *__restrict__ eta) {
    const int n = M.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ux = u[i], uy = u[n + i], uz = u[2 * n + i];
    double z = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = M.nbr[s * n + i];
        const int k = s * n + i;
        z += M.bx[k] * (ux + u[j]) + M.by[k] * (uy + u[n + j]) + M.bz[k] * (uz + u[2 * n + j]);
    }
    eta[i] = z + M.cor[i];
}

__global__ void __launch_bounds__(kBlock) k_rhs(DevMesh M, const double *__restrict__ u,
                                                const double *__restrict__ lu,
                                                double *__restrict__ f) {
    const int n = M.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = M.g;
    const double ux = u[i], uy = u[n + i], uz = u[2 * n + i], h = u[3 * n + i];
    const double Ei = 0.5 * (ux * ux + uy * uy + uz * uz) + g * h;
    const double l0 = lu[i], l1 = lu[n + i], l2 = lu[2 * n + i], l3 = lu[3 * n + i];
    double gx = 0.0, gy = 0.0, gz = 0.0, dv = 0.0, zt = 0.0;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = M.nbr[s * n + i];
        const int k = s * n + i;
        const double vx = u[j], vy = u[n + j], vz = u[2 * n + j], hj = u[3 * n + j];
        const double ax = M.ax[k], ay = M.ay[k], az = M.az[k];
        const double Ej = 0.5 * (vx * vx + vy * vy + vz * vz) + g * hj;
        const double dE = Ej - Ei;
        gx += ax * dE;
        gy += ay * dE;
        gz += az * dE;
        dv += ax * (h * ux + hj * vx) + ay * (h * uy + hj * vy) + az * (h * uz + hj * vz);
        zt += M.bx[k] * (ux + vx) + M.by[k] * (uy + vy) + M.bz[k] * (uz + vz);
        const double c = M.cl[k];
        d0 += c * (lu[j] - l0);
        d1 += c * (lu[n + j] - l1);
        d2 += c * (lu[2 * n + j] - l2);
        d3 += c * (lu[3 * n + j] - l3);
    }
    const double nx = M.nx[i], ny = M.ny[i], nz = M.nz[i];
    const double gr = nx * gx + ny * gy + nz * gz;       // tangent projection of grad E
    gx -= gr * nx;
    gy -= gr * ny;
    gz -= gr * nz;
    const double eta = zt + M.cor[i];
    const double px = ny * uz - nz * uy, py = nz * ux - nx * uz, pz = nx * uy - ny * ux;
    const double nu = M.nu;
    f[i] = -eta * px - gx - nu * d0;
    f[n + i] = -eta * py - gy - nu * d1;
    f[2 * n + i] = -eta * pz - gz - nu * d2;
    f[3 * n + i] = -dv - nu * d3;
}

// out = dt*scale*J(u) x + sum_k c_k v_k, with optional reduction epilogue.
template <int EPI>
__global__ void __launch_bounds__(kBlock) k_jv(DevMesh M, JvArgs a) {
    __shared__ double lds[16];
    if (EPI == kEpiIom2) {
        if (a.ctl->brk != 0 || a.ctl->beta_zero) return;
    }
    const int n = M.n;
    const double g = M.g, nu = M.nu;
    const double sc = a.dt * (a.scale_ptr ? *a.scale_ptr : 1.0);
    double cax[kPmax];
#pragma unroll
    for (int k = 0; k < kPmax; ++k) cax[k] = (k < a.naxpy) ? *a.axc[k] : 0.0;
    const double *__restrict__ u = a.u;
    const double *__restrict__ x = a.x;
    const double *__restrict__ lx = a.lx;
    double r0 = 0.0, r1 = 0.0;   // reduction partials
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ux = u[i], uy = u[n + i], uz = u[2 * n + i], uh = u[3 * n + i];
        const double xx = x[i], xy = x[n + i], xz = x[2 * n + i], xh = x[3 * n + i];
        const double l0 = lx[i], l1 = lx[n + i], l2 = lx[2 * n + i], l3 = lx[3 * n + i];
        const double si = ux * xx + uy * xy + uz * xz + g * xh;       // u.x_vel + g x_h
        const double fx = uh * xx + xh * ux, fy = uh * xy + xh * uy, fz = uh * xz + xh * uz;
        double gx = 0.0, gy = 0.0, gz = 0.0, dv = 0.0, zt = 0.0;
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int j = M.nbr[s * n + i];
            const int k = s * n + i;
            const double vx = x[j], vy = x[n + j], vz = x[2 * n + j], vh = x[3 * n + j];
            const double wx = u[j], wy = u[n + j], wz = u[2 * n + j], wh = u[3 * n + j];
            const double ax = M.ax[k], ay = M.ay[k], az = M.az[k];
            const double sj = wx * vx + wy * vy + wz * vz + g * vh;
            const double ds = sj - si;
            gx += ax * ds;
            gy += ay * ds;
            gz += az * ds;
            dv += ax * (fx + (wh * vx + vh * wx)) + ay * (fy + (wh * vy + vh * wy)) +
                  az * (fz + (wh * vz + vh * wz));
            zt += M.bx[k] * (xx + vx) + M.by[k] * (xy + vy) + M.bz[k] * (xz + vz);
            const double c = M.cl[k];
            d0 += c * (lx[j] - l0);
            d1 += c * (lx[n + j] - l1);
            d2 += c * (lx[2 * n + j] - l2);
            d3 += c * (lx[3 * n + j] - l3);
        }
        const double nx = M.nx[i], ny = M.ny[i], nz = M.nz[i];
        const double gr = nx * gx + ny * gy + nz * gz;
        gx -= gr * nx;
        gy -= gr * ny;
        gz -= gr * nz;
        const double eta = a.eta[i];
        // J_v x: -(V.x) (n x u);  J_r x: -eta (n x x) - nu L^2 x;  J_m x: -G(u.x + g x_h), -D(h x + x_h u)
        const double pux = ny * uz - nz * uy, puy = nz * ux - nx * uz, puz = nx * uy - ny * ux;
        const double pxx = ny * xz - nz * xy, pxy = nz * xx - nx * xz, pxz = nx * xy - ny * xx;
        double o0 = sc * (-zt * pux - eta * pxx - gx - nu * d0);
        double o1 = sc * (-zt * puy - eta * pxy - gy - nu * d1);
        double o2 = sc * (-zt * puz - eta * pxz - gz - nu * d2);
        double o3 = sc * (-dv - nu * d3);
#pragma unroll
        for (int k = 0; k < kPmax; ++k) {
            if (k < a.naxpy) {
                const double *v = a.axv[k];
                o0 += cax[k] * v[i];
                o1 += cax[k] * v[n + i];
                o2 += cax[k] * v[2 * n + i];
                o3 += cax[k] * v[3 * n + i];
            }
        }
        a.out[i] = o0;
        a.out[n + i] = o1;
        a.out[2 * n + i] = o2;
        a.out[3 * n + i] = o3;
        if (EPI == kEpiIom2) {
            const double *rj = a.rj;
            r0 += o0 * rj[i] + o1 * rj[n + i] + o2 * rj[2 * n + i] + o3 * rj[3 * n + i];
            if (a.rjm1) {
                const double *rm = a.rjm1;
                r1 += o0 * rm[i] + o1 * rm[n + i] + o2 * rm[2 * n + i] + o3 * rm[3 * n + i];
            }
        } else if (EPI == kEpiNorm) {
            r0 += o0 * o0 + o1 * o1 + o2 * o2 + o3 * o3;
        }
    }
    if (EPI == kEpiNone) return;
    double v[2] = {r0, r1};
    block_sum<2>(v, lds);
    uint32_t *ctr = &a.ctl->counters[EPI == kEpiIom2 ? 0 : 1];
    if (!grid_arrive<2>(v, a.partials, ctr)) return;
    double tot[2];
    grid_finish<2>(tot, a.partials, ctr, lds);
    if (threadIdx.x == 0) {
        PhiCtl *c = a.ctl;
        if (EPI == kEpiIom2) {
            const int j = a.j;
            c->H[j * kMmax + j] = c->sigma[j] * tot[0];
            if (j > 0) c->H[(j - 1) * kMmax + j] = c->sigma[j - 1] * tot[1];
        } else {
            const double beta = sqrt(tot[0]);
            c->beta = beta;
            c->beta_zero = (beta == 0.0) ? 1 : 0;
            c->sigma[0] = beta > 0.0 ? 1.0 / beta : 0.0;
            c->brk = 0;
        }
    }
}

}  // namespace

void launch_lap4(const DevMesh &M, const double *psi, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_lap4, dim3(grid_for(M.n)), dim3(kBlock), 0, s, M, psi, out);
}

void launch_linearize(const DevMesh &M, const double *u, double *eta, hipStream_t s) {
    hipLaunchKernelGGL(k_linearize, dim3(grid_for(M.n)), dim3(kBlock), 0, s, M, u, eta);
}

void launch_rhs(const DevMesh &M, const double *u, const double *lu, double *f, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(M.n)), dim3(kBlock), 0, s, M, u, lu, f);
}

void launch_jv(const DevMesh &M, const JvArgs &a, int epi, hipStream_t s) {
    if (epi == kEpiNone)
        hipLaunchKernelGGL(k_jv<kEpiNone>, dim3(grid_for(M.n)), dim3(kBlock), 0, s, M, a);
    else if (epi == kEpiIom2)
        hipLaunchKernelGGL(k_jv<kEpiIom2>, dim3(grid_capped(M.n)), dim3(kBlock), 0, s, M, a);
    else
        hipLaunchKernelGGL(k_jv<kEpiNorm>, dim3(grid_capped(M.n)), dim3(kBlock), 0, s, M, a);
}

}  // namespace xrb
