// Finite-volume stencil kernels of the shallow-water model (Sec. 2):
//   F(u)    eq. sweqsinv with D_f = -nu L^2 (eq. swdis)
//   J(u) x  eqs. dynjs-dynjc, fused with the IOM2 dot products or the w_j
//           recurrence axpys of Alg. 1
//
// Edge-parallel mapping: eight consecutive lanes serve one cell, lane s < 6
// handling the edge to neighbour slot s (lanes 6 and 7 carry zero weights).
// Each lane gathers its neighbour, forms its edge terms, and a fixed DPP
// butterfly over the eight lanes sums them (bitwise identical in all eight).
// This gives eight times the memory-level parallelism of one thread per
// cell, which the small grids need.  The two-ring dissipation stencil
// L(L x) takes L x from a preceding one-ring pass (launch_lap4).
#include "reduce.h"
#include "xrb_internal.h"

namespace xrb {

namespace {

constexpr int kLanes = 8;

inline int cells_grid(int n, int block) {
    const int cpb = block / kLanes;
    int g = (n + cpb - 1) / cpb;
    return g < 1 ? 1 : g;
}

// Lane exchange inside a row by a DPP control word (VALU, no LDS traffic).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the eight lanes of a cell: half-row mirror (lane i with 7-i),
// then xor 1 and xor 2 inside each quad.  Every lane ends with the same
// operands added in the same pairs (only commuted), so the eight results
// are bitwise identical.
__device__ inline double grp_sum(double v) {
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    return v;
}

// Cell record: unit centre and Coriolis parameter, two 16-byte loads.
struct Cell {
    double x, y, z, f;
};
__device__ inline Cell load_cell(const double *__restrict__ cen, int i) {
    const double2 *p = reinterpret_cast<const double2 *>(cen) + 2 * (size_t)i;
    const double2 a = p[0], b = p[1];
    return {a.x, a.y, b.x, b.y};
}

// Flux and circulation weights of the edge i -> j rebuilt from its two
// scalars: a = alpha (x_j - x_i), b = beta (x_i x x_j).  Lanes without an
// edge pass alpha = beta = 0.
struct EdgeW {
    double ax, ay, az, bx, by, bz;
};
__device__ inline EdgeW edge_weights(const Cell &ci, const Cell &cj, double al, double be) {
    EdgeW w;
    w.ax = al * (cj.x - ci.x);
    w.ay = al * (cj.y - ci.y);
    w.az = al * (cj.z - ci.z);
    w.bx = be * (ci.y * cj.z - ci.z * cj.y);
    w.by = be * (ci.z * cj.x - ci.x * cj.z);
    w.bz = be * (ci.x * cj.y - ci.y * cj.x);
    return w;
}

// first cell of this thread's group and the stride, in cells
__device__ inline int cell0() { return (int)((blockIdx.x * blockDim.x + threadIdx.x) / kLanes); }
__device__ inline int cell_stride() { return (int)((gridDim.x * blockDim.x) / kLanes); }

__global__ void __launch_bounds__(256) k_lap4(DevMesh M, const double *__restrict__ psi,
                                              double *__restrict__ out, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    psi = member_ptr(psi, bt.ws, mk);
    out = member_ptr(out, bt.ws, mk);
    const int n = M.n;
    const int s = threadIdx.x & (kLanes - 1);
    for (int i = cell0(); i < n; i += cell_stride()) {
        const int e = 6 * i + (s < 6 ? s : 0);
        const int j = s < 6 ? M.nbr[e] : i;
        const double c = s < 6 ? M.cl[e] : 0.0;
        double a[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) a[b] = grp_sum(c * (psi[b * n + j] - psi[b * n + i]));
        if (s < 4) out[s * n + i] = a[s];
    }
}

__global__ void __launch_bounds__(256) k_linearize(DevMesh M, const double *__restrict__ u,
                                                   double *__restrict__ eta, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    u = member_ptr(u, bt.ws, mk);
    eta = member_ptr(eta, bt.ws, mk);
    const int n = M.n;
    const int s = threadIdx.x & (kLanes - 1);
    for (int i = cell0(); i < n; i += cell_stride()) {
        const bool edge = s < 6;
        const int e = 6 * i + (edge ? s : 0);
        const int j = edge ? M.nbr[e] : i;
        const Cell ci = load_cell(M.cen, i), cj = load_cell(M.cen, j);
        const EdgeW w = edge_weights(ci, cj, 0.0, edge ? M.beta[e] : 0.0);
        double z = w.bx * (u[i] + u[j]) + w.by * (u[n + i] + u[n + j]) +
                   w.bz * (u[2 * n + i] + u[2 * n + j]);
        z = grp_sum(z);
        if (s == 0) eta[i] = z + ci.f;
    }
}

__global__ void __launch_bounds__(256) k_rhs(DevMesh M, const double *__restrict__ u,
                                             const double *__restrict__ lu,
                                             double *__restrict__ f, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    u = member_ptr(u, bt.ws, mk);
    lu = member_ptr(lu, bt.ws, mk);
    f = member_ptr(f, bt.ws, mk);
    const int n = M.n;
    const double g = M.g;
    const int s = threadIdx.x & (kLanes - 1);
    for (int i = cell0(); i < n; i += cell_stride()) {
        const bool edge = s < 6;
        const int e = 6 * i + (edge ? s : 0);
        const int j = edge ? M.nbr[e] : i;
        const double ux = u[i], uy = u[n + i], uz = u[2 * n + i], h = u[3 * n + i];
        const double vx = u[j], vy = u[n + j], vz = u[2 * n + j], hj = u[3 * n + j];
        const Cell ci = load_cell(M.cen, i), cj = load_cell(M.cen, j);
        const EdgeW w = edge_weights(ci, cj, edge ? M.alpha[e] : 0.0, edge ? M.beta[e] : 0.0);
        const double ax = w.ax, ay = w.ay, az = w.az, bx = w.bx, by = w.by, bz = w.bz;
        const double c = edge ? M.cl[e] : 0.0;
        const double Ei = 0.5 * (ux * ux + uy * uy + uz * uz) + g * h;
        const double Ej = 0.5 * (vx * vx + vy * vy + vz * vz) + g * hj;
        const double dE = Ej - Ei;
        const double gx = grp_sum(ax * dE), gy0 = grp_sum(ay * dE), gz0 = grp_sum(az * dE);
        const double dv = grp_sum(ax * (h * ux + hj * vx) + ay * (h * uy + hj * vy) +
                                  az * (h * uz + hj * vz));
        const double zt = grp_sum(bx * (ux + vx) + by * (uy + vy) + bz * (uz + vz));
        double d[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = grp_sum(c * (lu[b * n + j] - lu[b * n + i]));
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double gr = nx * gx + ny * gy0 + nz * gz0;       // tangent projection of grad E
        const double Gx = gx - gr * nx, Gy = gy0 - gr * ny, Gz = gz0 - gr * nz;
        const double eta = zt + ci.f;
        const double px = ny * uz - nz * uy, py = nz * ux - nx * uz, pz = nx * uy - ny * ux;
        const double nu = M.nu;
        double o[4];
        o[0] = -eta * px - Gx - nu * d[0];
        o[1] = -eta * py - Gy - nu * d[1];
        o[2] = -eta * pz - Gz - nu * d[2];
        o[3] = -dv - nu * d[3];
        if (s < 4) f[s * n + i] = o[s];
    }
}

// out = dt*J(u) x + sum_k c_k v_k, with an optional reduction epilogue
// (IOM2: raw dot partials; recurrence: norm partials).
template <int EPI>
__global__ void __launch_bounds__(256) k_jv(DevMesh M, JvArgs a, Batch bt) {
    __shared__ double lds[64];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const double g = M.g, nu = M.nu;
    const double sc = bt.dtk ? bt.dtk[mk] : a.dt;
    const int s = threadIdx.x & (kLanes - 1);
    double cax[kPmax];
    const double *axv[kPmax];
#pragma unroll
    for (int k = 0; k < kPmax; ++k) {
        cax[k] = (k < a.naxpy) ? *ctl_field(a.axc[k], mk) : 0.0;
        axv[k] = (k < a.naxpy) ? member_ptr(a.axv[k], bt.ws, mk) : nullptr;
    }
    const double *__restrict__ u = member_ptr(a.u, bt.ws, mk);
    const double *__restrict__ x = member_ptr(a.x, bt.ws, mk);
    const double *__restrict__ lx = member_ptr(a.lx, bt.ws, mk);
    const double *__restrict__ etak = member_ptr(a.eta, bt.ws, mk);
    double *__restrict__ outk = member_ptr(a.out, bt.ws, mk);
    const double *__restrict__ rjm1 = member_ptr(a.rjm1, bt.ws, mk);
    double r0 = 0.0, r1 = 0.0;   // this lane's reduction partials
    for (int i = cell0(); i < n; i += cell_stride()) {
        const bool edge = s < 6;
        const int e = 6 * i + (edge ? s : 0);
        const int j = edge ? M.nbr[e] : i;
        const double ux = u[i], uy = u[n + i], uz = u[2 * n + i], uh = u[3 * n + i];
        const double xx = x[i], xy = x[n + i], xz = x[2 * n + i], xh = x[3 * n + i];
        const double vx = x[j], vy = x[n + j], vz = x[2 * n + j], vh = x[3 * n + j];
        const double wx = u[j], wy = u[n + j], wz = u[2 * n + j], wh = u[3 * n + j];
        const Cell ci = load_cell(M.cen, i), cj = load_cell(M.cen, j);
        const EdgeW w = edge_weights(ci, cj, edge ? M.alpha[e] : 0.0, edge ? M.beta[e] : 0.0);
        const double ax = w.ax, ay = w.ay, az = w.az, bx = w.bx, by = w.by, bz = w.bz;
        const double c = edge ? M.cl[e] : 0.0;
        const double si = ux * xx + uy * xy + uz * xz + g * xh;       // u.x_vel + g x_h
        const double sj = wx * vx + wy * vy + wz * vz + g * vh;
        const double ds = sj - si;
        const double fx = uh * xx + xh * ux, fy = uh * xy + xh * uy, fz = uh * xz + xh * uz;
        const double gx = grp_sum(ax * ds), gy0 = grp_sum(ay * ds), gz0 = grp_sum(az * ds);
        const double dv = grp_sum(ax * (fx + (wh * vx + vh * wx)) + ay * (fy + (wh * vy + vh * wy)) +
                                  az * (fz + (wh * vz + vh * wz)));
        const double zt = grp_sum(bx * (xx + vx) + by * (xy + vy) + bz * (xz + vz));
        double d[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = grp_sum(c * (lx[b * n + j] - lx[b * n + i]));
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double gr = nx * gx + ny * gy0 + nz * gz0;
        const double Gx = gx - gr * nx, Gy = gy0 - gr * ny, Gz = gz0 - gr * nz;
        const double eta = etak[i];
        // J_v x: -(V.x) (n x u);  J_r x: -eta (n x x) - nu L^2 x;
        // J_m x: -G(u.x + g x_h), -D(h x + x_h u)
        const double pux = ny * uz - nz * uy, puy = nz * ux - nx * uz, puz = nx * uy - ny * ux;
        const double pxx = ny * xz - nz * xy, pxy = nz * xx - nx * xz, pxz = nx * xy - ny * xx;
        double o[4];
        o[0] = sc * (-zt * pux - eta * pxx - Gx - nu * d[0]);
        o[1] = sc * (-zt * puy - eta * pxy - Gy - nu * d[1]);
        o[2] = sc * (-zt * puz - eta * pxz - Gz - nu * d[2]);
        o[3] = sc * (-dv - nu * d[3]);
        if (s < 4) {
            const int oi = s * n + i;
            double ob = o[s];
#pragma unroll
            for (int k = 0; k < kPmax; ++k)
                if (k < a.naxpy) ob += cax[k] * axv[k][oi];
            outk[oi] = ob;
            if (EPI == kEpiIom2) {
                const double xs = s == 0 ? xx : (s == 1 ? xy : (s == 2 ? xz : xh));
                r0 += ob * xs;
                if (rjm1) r1 += ob * rjm1[oi];
            } else if (EPI == kEpiNorm) {
                r0 += ob * ob;
            }
        }
    }
    if (EPI == kEpiIom2) {
        double v[2] = {r0, r1};
        block_sum_all<2>(v, lds);
        put_partials<2>(v, a.dot_out + (size_t)mk * kPartStride);
    } else if (EPI == kEpiNorm) {
        double v[1] = {r0};
        block_sum_all<1>(v, lds);
        put_partials<1>(v, a.nrm_out + (size_t)mk * kPartStride);
    }
}

}  // namespace

void launch_lap4(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_lap4, dim3(cells_grid(M.n, 256), b.nm), dim3(256), 0, s, M, psi, out, b);
}

void launch_linearize(const DevMesh &M, const double *u, double *eta, const Batch &b,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_linearize, dim3(cells_grid(M.n, 256), b.nm), dim3(256), 0, s, M, u, eta, b);
}

void launch_rhs(const DevMesh &M, const double *u, const double *lu, double *f, const Batch &b,
                hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(cells_grid(M.n, 256), b.nm), dim3(256), 0, s, M, u, lu, f, b);
}

int launch_jv(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    if (epi == kEpiNone) {
        hipLaunchKernelGGL(k_jv<kEpiNone>, dim3(cells_grid(M.n, 256), b.nm), dim3(256), 0, s, M, a,
                           b);
        return 0;
    }
    const int grid = red_parts(M.n);
    if (epi == kEpiIom2)
        hipLaunchKernelGGL(k_jv<kEpiIom2>, dim3(grid, b.nm), dim3(256), 0, s, M, a, b);
    else
        hipLaunchKernelGGL(k_jv<kEpiNorm>, dim3(grid, b.nm), dim3(256), 0, s, M, a, b);
    return grid;
}

}  // namespace xrb
