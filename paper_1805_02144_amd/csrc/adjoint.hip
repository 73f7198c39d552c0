// Kernels of the adjoint (vector-Jacobian product) path.  The paper has no
// adjoint; this is the continuous adjoint of the phi-combination ODE (eq.
// 3.15) on the substeps of its forward solve:
//   mu' = -A^T mu backwards from the output cotangents, vbar_j the moments
//   int mu t^(j-1)/(j-1)! dt, and the A-term int K(mu, y) dt, where
//   K(a, b) = grad_u <a, J(u) b>.
//
//   k_lapT    L^T psi on four fields (prepass of the two-ring (L^T)^2;
//             k_lapT_lds on grids with chunk tables)
//   k_jtv     dt J(u)^T x (+ axpys) with the IOM2 / norm epilogues of k_jv,
//             so the IOM2 driver builds a Krylov space of A^T unchanged
//             (k_jtv_lds: its form on grids with chunk tables)
//   k_kpairs  acc += sum_r c_r K(a_r, b_r) (k_kpairs_lds on grids with
//             chunk tables)
//   k_lincomb_multi  several combinations of one contiguous basis at once
//   k_zgemm   Z_r = sum_c z_rc What_c (the forward substep's solution basis)
//   k_adj_gexp    finishes the last IOM2 column, exp(tau G) of the adjoint
//                 augmented matrix, the error ratio and the combination
//                 coefficients of mu_k and the moments
//   k_adj_vanloan exp of the Van Loan block matrix and the Z coefficients
//
// Transposes in gather form: with rho_ij = A_i / A_j and the weights of the
// forward stencils (a = alpha (x_j - x_i), b = beta (x_i x x_j), c = l/(dA)),
//   (V^T s)_i = A_i sum b_ij (s_i/A_i - s_j/A_j)
//   (G^T w)_i = -A_i sum a_ij . (P_i w_i/A_i + P_j w_j/A_j)
//   (D^T p)_i = A_i sum a_ij (p_i/A_i - p_j/A_j)
//   (L^T p)_i = A_i sum c_ij (p_j/A_j - p_i/A_i)
// (a_ji = -a_ij A_i/A_j and b_ji = -b_ij A_i/A_j, c_ji = c_ij A_i/A_j.)
#include "column.h"
#include "reduce.h"
#include "stencil_common.h"
#include "xrb_internal.h"

namespace xrb {
namespace {

using namespace stc;

template <int L>
__global__ void __launch_bounds__(256) k_lapT(DevMesh M, const double *__restrict__ psi,
                                              double *__restrict__ out, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    psi = member_ptr(psi, bt.ws, mk);
    out = member_ptr(out, bt.ws, mk);
    const int n = M.n;
    const int q = threadIdx.x & (L - 1);
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        const Cell ci = load_cell(M.cen, i);
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        double pi[4];
        load4(psi, i, pi);
#pragma unroll
        for (int s = q; s < 6; s += L) {
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            const double c = M.cl[e];
            const double raj = M.cen[4 * (size_t)j + 3];
            double pj[4];
            load4(psi, j, pj);
#pragma unroll
            for (int b = 0; b < 4; ++b) a[b] += c * (pj[b] * raj - pi[b] * ci.ra);
        }
        const double Ai = 1.0 / ci.ra;
#pragma unroll
        for (int b = 0; b < 4; ++b) a[b] = grp_sum<L>(a[b]);
#pragma unroll
        for (int b = q; b < 4; b += L) out[4 * i + b] = Ai * a[b];
    }
}

// k_lapT on grids with chunk tables: the chunk's cells and their one-ring
// halo staged in LDS as psi ra (ra = 1/A), then
// (L^T psi)_i = A_i sum_s c_s ((psi ra)_j - (psi ra)_i) with two lanes per
// cell.  Any grid that is a multiple of the XCD count.
constexpr int kLapTLdsL = 2;
constexpr int kLapTLdsBlock = kChunk * kLapTLdsL;

__global__ void __launch_bounds__(kLapTLdsBlock) k_lapT_lds(DevMesh M, const double *__restrict__ psi,
                                                             double *__restrict__ out, Batch bt) {
    constexpr int L = kLapTLdsL, C = kChunk, HM = kHaloMax;
    __shared__ double2 sx[(C + HM) * 2];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const double2 *x2 = reinterpret_cast<const double2 *>(member_ptr(psi, bt.ws, mk));
    out = member_ptr(out, bt.ws, mk);
    const Halo &h = M.halo;
    const int n = M.n;
    const int t = threadIdx.x, q = t & (L - 1);
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nbx = G / kXcd, xcd = b % kXcd, kk = b / kXcd;
    const ChunkSpan span = xcd_chunks(h.nchunks, xcd);
    const int ck_end = span.end;
    for (int ck = span.first + kk; ck < ck_end; ck += nbx) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        const int h0 = h.hoff[ck], hn = h.hoff[ck + 1] - h0;
        __syncthreads();   // the previous chunk's readers are done
        for (int k = t; k < 2 * (cnt + hn); k += kLapTLdsBlock) {
            const int m = k >> 1;
            const int j = m < cnt ? c0 + m : h.hids[h0 + (m - cnt)];
            const double ra = M.cen[4 * (size_t)j + 3];
            const double2 v = x2[2 * (size_t)j + (k & 1)];
            sx[(m < cnt ? 2 * m : 2 * (C + m - cnt)) + (k & 1)] = make_double2(v.x * ra, v.y * ra);
        }
        __syncthreads();
        const int li = t / L;
        if (li >= cnt) continue;
        const int i = c0 + li;
        const double2 a0 = sx[2 * li], a1 = sx[2 * li + 1];
        const double pi[4] = {a0.x, a0.y, a1.x, a1.y};
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int e = 6 * i + slot_of<L>(q, k);
            const int lj = h.lnbr[e];
            const double c = M.cl[e];
            const double2 b0 = sx[2 * lj], b1 = sx[2 * lj + 1];
            const double pj[4] = {b0.x, b0.y, b1.x, b1.y};
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) acc[bb] = fma(c, pj[bb] - pi[bb], acc[bb]);
        }
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[bb] = grp_sum<L>(acc[bb]);
        const double Ai = 1.0 / M.cen[4 * (size_t)i + 3];
#pragma unroll
        for (int k = 0; k < kCompIter<L>; ++k) out[4 * i + comp_of<L>(q, k)] = Ai * acc[comp_of<L>(q, k)];
    }
}

// out = dt J(u)^T x + sum_k c_k v_k.  J^T x (the transpose of k_jv's
// product):
//   velocity: -V^T(x . (n x u)) + eta (n x x) - (G^T x_vel) u - h D^T x_h
//             - nu (L^T)^2 x_vel
//   depth:    -g G^T x_vel - (D^T x_h) . u - nu (L^T)^2 x_h
// Threads per block at most, as for the forward product: plain and norm 256,
// IOM2 1024 (the smaller bound leaves registers enough to avoid spills).
template <int EPI>
constexpr int kJtvMaxBlock = EPI == kEpiIom2 ? 1024 : 256;

template <int EPI, int L>
__global__ void __launch_bounds__(kJtvMaxBlock<EPI>) k_jtv(DevMesh M, JvArgs a, Batch bt) {
    __shared__ double lds[64];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const double g = M.g, nu = M.nu;
    const double sc = bt.dtk ? bt.dtk[mk] : a.dt;
    const int q = threadIdx.x & (L - 1);
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
    double r0 = 0.0, r1 = 0.0;
    // several passes per block: sweep each XCD's cells window by window
    for (CellRange r = block_cells_swept<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        double ui[4], xi[4], lxi[4];
        load4(u, i, ui);
        load4(x, i, xi);
        load4(lx, i, lxi);
        const double ux = ui[0], uy = ui[1], uz = ui[2], uh = ui[3];
        const double xx = xi[0], xy = xi[1], xz = xi[2], xh = xi[3];
        const Cell ci = load_cell(M.cen, i);
        const double nx = ci.x, ny = ci.y, nz = ci.z, rai = ci.ra;
        // s_i = x_i . (n_i x u_i), P_i x_i
        const double si = xx * (ny * uz - nz * uy) + xy * (nz * ux - nx * uz) + xz * (nx * uy - ny * ux);
        const double xn = nx * xx + ny * xy + nz * xz;
        const double tx = xx - xn * nx, ty = xy - xn * ny, tz = xz - xn * nz;
        double vsx = 0.0, vsy = 0.0, vsz = 0.0, gq = 0.0, drx = 0.0, dry = 0.0, drz = 0.0;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll(2)
        for (int s = q; s < 6; s += L) {
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            double xj[4], uj[4], lxj[4];
            load4(x, j, xj);
            load4(u, j, uj);
            load4(lx, j, lxj);
            const double vx = xj[0], vy = xj[1], vz = xj[2], vh = xj[3];
            const double wx = uj[0], wy = uj[1], wz = uj[2];
            const Cell cj = load_cell(M.cen, j);
            const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
            const double c = M.cl[e];
            const double raj = cj.ra;
            const double sj = vx * (cj.y * wz - cj.z * wy) + vy * (cj.z * wx - cj.x * wz) +
                              vz * (cj.x * wy - cj.y * wx);
            const double vn = cj.x * vx + cj.y * vy + cj.z * vz;
            const double px = vx - vn * cj.x, py = vy - vn * cj.y, pz = vz - vn * cj.z;
            const double ds = si * rai - sj * raj;
            vsx += w.bx * ds;
            vsy += w.by * ds;
            vsz += w.bz * ds;
            gq += w.ax * (tx * rai + px * raj) + w.ay * (ty * rai + py * raj) + w.az * (tz * rai + pz * raj);
            const double dh = xh * rai - vh * raj;
            drx += w.ax * dh;
            dry += w.ay * dh;
            drz += w.az * dh;
#pragma unroll
            for (int b = 0; b < 4; ++b) d[b] += c * (lxj[b] * raj - lxi[b] * rai);
        }
        vsx = grp_sum<L>(vsx);
        vsy = grp_sum<L>(vsy);
        vsz = grp_sum<L>(vsz);
        gq = grp_sum<L>(gq);
        drx = grp_sum<L>(drx);
        dry = grp_sum<L>(dry);
        drz = grp_sum<L>(drz);
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = grp_sum<L>(d[b]);
        const double Ai = 1.0 / rai;
        const double qq = -Ai * gq;                              // (G^T x_vel)_i
        const double rx = Ai * drx, ry = Ai * dry, rz = Ai * drz;  // (D^T x_h)_i
        const double eta = etak[i];
        double o[4];
        o[0] = sc * (-Ai * vsx + eta * (ny * xz - nz * xy) - qq * ux - uh * rx - nu * Ai * d[0]);
        o[1] = sc * (-Ai * vsy + eta * (nz * xx - nx * xz) - qq * uy - uh * ry - nu * Ai * d[1]);
        o[2] = sc * (-Ai * vsz + eta * (nx * xy - ny * xx) - qq * uz - uh * rz - nu * Ai * d[2]);
        o[3] = sc * (-g * qq - (rx * ux + ry * uy + rz * uz) - nu * Ai * d[3]);
        const double xs[4] = {xx, xy, xz, xh};
#pragma unroll
        for (int b = q; b < 4; b += L) {
            const int oi = 4 * i + b;
            double ob = o[b];
#pragma unroll
            for (int k = 0; k < kPmax; ++k)
                if (k < a.naxpy) ob += cax[k] * axv[k][oi];
            outk[oi] = ob;
            if (EPI == kEpiIom2) {
                r0 += ob * xs[b];
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

// k_jtv on grids with chunk tables, its neighbours staged in LDS like the
// forward k_jv_lds: for each chunk, one thread per cell of the chunk and of
// its one-ring halo loads the cell's x, u, L^T x and centre record and stores
// the area-scaled quantities its edges take -- s ra, (P x) ra, x_h ra and
// (L^T x) ra (s = x . (n x u), P x the tangential part of x_vel, ra = 1/A) --
// with the centre, 12 doubles; the chunk's own cells also keep u, x, eta and
// A.  Edge weights come from c and the chord (edge_weights_short), two lanes
// serve a cell, accumulations fuse.  Reductions as in k_jtv: per-lane
// partials, one block sum, the returned number of blocks.
constexpr int kJtvLdsL = 2;
constexpr int kJtvLdsBlock = kChunk * kJtvLdsL;

template <int EPI>
__global__ void __launch_bounds__(kJtvLdsBlock, 4) k_jtv_lds(DevMesh M, JvArgs a, Batch bt) {
    constexpr int L = kJtvLdsL, C = kChunk, S = kChunk + kHaloMax;
    // staged cells: (s ra, p_x ra) (p_y ra, p_z ra) (x_h ra, centre_x)
    // (centre_y, centre_z) ((L^T x)_0 ra, (L^T x)_1 ra) ((L^T x)_2 ra, (L^T x)_3 ra);
    // own cells: (u_x, u_y) (u_z, h) (x_x, x_y) (x_z, x_h) (eta, A)
    __shared__ double2 nA[S], nB[S], nC[S], nD[S], nE[S], nF[S];
    __shared__ double2 oU0[C], oU1[C], oX0[C], oX1[C], oE[C];
    __shared__ double lds[64];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const double g = M.g, nu = M.nu;
    const double sc = bt.dtk ? bt.dtk[mk] : a.dt;
    double cax[kPmax];
    const double *axv[kPmax];
#pragma unroll
    for (int k = 0; k < kPmax; ++k) {
        cax[k] = (k < a.naxpy) ? *ctl_field(a.axc[k], mk) : 0.0;
        axv[k] = (k < a.naxpy) ? member_ptr(a.axv[k], bt.ws, mk) : nullptr;
    }
    const double2 *x2 = reinterpret_cast<const double2 *>(member_ptr(a.x, bt.ws, mk));
    const double2 *u2 = reinterpret_cast<const double2 *>(member_ptr(a.u, bt.ws, mk));
    const double2 *l2 = reinterpret_cast<const double2 *>(member_ptr(a.lx, bt.ws, mk));
    const double2 *c2 = reinterpret_cast<const double2 *>(M.cen);
    const double *__restrict__ etak = member_ptr(a.eta, bt.ws, mk);
    double *__restrict__ outk = member_ptr(a.out, bt.ws, mk);
    // column 0 has no R_{-1}: its second dot runs against x and is not used
    const double *__restrict__ rjm1 = member_ptr(a.rjm1 ? a.rjm1 : a.x, bt.ws, mk);
    const Halo &h = M.halo;
    const int t = threadIdx.x;
    const int q = t & (L - 1);
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nbx = G / kXcd, xcd = b % kXcd, kk = b / kXcd;
    const ChunkSpan span = xcd_chunks(h.nchunks, xcd);
    const int ck_end = span.end;
    double r0 = 0.0, r1 = 0.0;
    for (int ck = span.first + kk; ck < ck_end; ck += nbx) {
        const int c0 = ck * C;
        const int cnt = min(C, n - c0);
        const int h0 = h.hoff[ck], hn = h.hoff[ck + 1] - h0;
        __syncthreads();   // the previous chunk's readers are done
        for (int m = t; m < cnt + hn; m += kJtvLdsBlock) {
            const bool own = m < cnt;
            const int j = own ? c0 + m : h.hids[h0 + (m - cnt)];
            const int sl = own ? m : C + (m - cnt);
            const double2 v0 = x2[2 * (size_t)j], v1 = x2[2 * (size_t)j + 1];
            const double2 w0 = u2[2 * (size_t)j], w1 = u2[2 * (size_t)j + 1];
            const double2 e0 = c2[2 * (size_t)j], e1 = c2[2 * (size_t)j + 1];
            const double2 l0 = l2[2 * (size_t)j], l1 = l2[2 * (size_t)j + 1];
            const double vx = v0.x, vy = v0.y, vz = v1.x, vh = v1.y;
            const double wx = w0.x, wy = w0.y, wz = w1.x;
            const double cx = e0.x, cy = e0.y, cz = e1.x, ra = e1.y;
            const double sj = vx * (cy * wz - cz * wy) + vy * (cz * wx - cx * wz) + vz * (cx * wy - cy * wx);
            const double vn = cx * vx + cy * vy + cz * vz;
            nA[sl] = make_double2(sj * ra, (vx - vn * cx) * ra);
            nB[sl] = make_double2((vy - vn * cy) * ra, (vz - vn * cz) * ra);
            nC[sl] = make_double2(vh * ra, cx);
            nD[sl] = make_double2(cy, cz);
            nE[sl] = make_double2(l0.x * ra, l0.y * ra);
            nF[sl] = make_double2(l1.x * ra, l1.y * ra);
            if (own) {
                oU0[m] = w0;
                oU1[m] = w1;
                oX0[m] = v0;
                oX1[m] = v1;
                oE[m] = make_double2(etak[j], 1.0 / ra);
            }
        }
        __syncthreads();
        const int li = t / L;
        if (li >= cnt) continue;
        const int i = c0 + li;
        const double2 A0 = nA[li], B0 = nB[li], C0 = nC[li], D0 = nD[li], E0 = nE[li], F0 = nF[li];
        Cell ci;
        ci.x = C0.y;
        ci.y = D0.x;
        ci.z = D0.y;
        ci.ra = 0.0;
        const double Si = A0.x, tx = A0.y, ty = B0.x, tz = B0.y, Hi = C0.x;
        const double lxi[4] = {E0.x, E0.y, F0.x, F0.y};
        double vsx = 0.0, vsy = 0.0, vsz = 0.0, gq = 0.0, drx = 0.0, dry = 0.0, drz = 0.0;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int e = 6 * i + slot_of<L>(q, k);
            const int lj = h.lnbr[e];
            const double c = M.cl[e];
            const double2 Aj = nA[lj], Bj = nB[lj], Cj = nC[lj], Dj = nD[lj], Ej = nE[lj], Fj = nF[lj];
            Cell cj;
            cj.x = Cj.y;
            cj.y = Dj.x;
            cj.z = Dj.y;
            cj.ra = 0.0;
            const EdgeW w = edge_weights_short(ci, cj, c, M.half_r);
            const double ds = Si - Aj.x;
            vsx = fma(w.bx, ds, vsx);
            vsy = fma(w.by, ds, vsy);
            vsz = fma(w.bz, ds, vsz);
            gq = fma(w.az, tz + Bj.y, fma(w.ay, ty + Bj.x, fma(w.ax, tx + Aj.y, gq)));
            const double dh = Hi - Cj.x;
            drx = fma(w.ax, dh, drx);
            dry = fma(w.ay, dh, dry);
            drz = fma(w.az, dh, drz);
            const double lxj[4] = {Ej.x, Ej.y, Fj.x, Fj.y};
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) d[bb] = fma(c, lxj[bb] - lxi[bb], d[bb]);
        }
        vsx = grp_sum<L>(vsx);
        vsy = grp_sum<L>(vsy);
        vsz = grp_sum<L>(vsz);
        gq = grp_sum<L>(gq);
        drx = grp_sum<L>(drx);
        dry = grp_sum<L>(dry);
        drz = grp_sum<L>(drz);
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) d[bb] = grp_sum<L>(d[bb]);
        const double2 U0 = oU0[li], U1 = oU1[li], X0 = oX0[li], X1 = oX1[li], EE = oE[li];
        const double ux = U0.x, uy = U0.y, uz = U1.x, uh = U1.y;
        const double xx = X0.x, xy = X0.y, xz = X1.x, xh = X1.y;
        const double eta = EE.x, Ai = EE.y;
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double qq = -Ai * gq;                              // (G^T x_vel)_i
        const double rx = Ai * drx, ry = Ai * dry, rz = Ai * drz;  // (D^T x_h)_i
        double o[4];
        o[0] = sc * (-Ai * vsx + eta * (ny * xz - nz * xy) - qq * ux - uh * rx - nu * Ai * d[0]);
        o[1] = sc * (-Ai * vsy + eta * (nz * xx - nx * xz) - qq * uy - uh * ry - nu * Ai * d[1]);
        o[2] = sc * (-Ai * vsz + eta * (nx * xy - ny * xx) - qq * uz - uh * rz - nu * Ai * d[2]);
        o[3] = sc * (-g * qq - (rx * ux + ry * uy + rz * uz) - nu * Ai * d[3]);
        const double xs[4] = {xx, xy, xz, xh};
#pragma unroll
        for (int kc = 0; kc < kCompIter<L>; ++kc) {
            const int bb = comp_of<L>(q, kc);
            const int oi = 4 * i + bb;
            double ob = o[bb];
#pragma unroll
            for (int k = 0; k < kPmax; ++k)
                if (k < a.naxpy) ob += cax[k] * axv[k][oi];
            outk[oi] = ob;
            if (EPI == kEpiIom2) {
                r0 = fma(ob, xs[bb], r0);
                r1 = fma(ob, rjm1[oi], r1);
            } else if (EPI == kEpiNorm) {
                r0 = fma(ob, ob, r0);
            }
        }
    }
    if (EPI == kEpiNone) return;
    double *parts = (EPI == kEpiIom2 ? a.dot_out : a.nrm_out) + (size_t)mk * kPartStride;
    constexpr int NV = EPI == kEpiIom2 ? 2 : 1;
    double v[2] = {r0, r1};
    block_sum_all<2>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) parts[blockIdx.x * NV + k] = v[k];
}

// out (= or +=) scale * sum_{r < R} coef_r K(a_r, b_r), a_r = a0 + r sa,
// b_r = b0 + r sb.  K(a, b) = grad_u <a, J(u) b>:
//   velocity: -(V b)_i (a_i x n_i) + V^T(a . (b x n)) - (G^T a_vel)_i b_i
//             - b_h,i (D^T a_h)_i
//   depth:    -(D^T a_h)_i . b_i
template <int L>
__global__ void __launch_bounds__(256) k_kpairs(DevMesh M, KPairArgs k, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const int q = threadIdx.x & (L - 1);
    double *__restrict__ out = member_ptr(k.out, bt.ws, mk);
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        const Cell ci = load_cell(M.cen, i);
        const double nx = ci.x, ny = ci.y, nz = ci.z, rai = ci.ra;
        const double Ai = 1.0 / rai;
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        for (int pr = 0; pr < k.R; ++pr) {
            const double cr = k.scale * (k.coef ? k.coef[pr] : 1.0);
            if (cr == 0.0) continue;
            const double *__restrict__ av = member_ptr(k.a0, bt.ws, mk) + (size_t)pr * k.sa;
            const double *__restrict__ bv = member_ptr(k.b0, bt.ws, mk) + (size_t)pr * k.sb;
            double ai_[4], bi_[4];
            load4(av, i, ai_);
            load4(bv, i, bi_);
            const double ax = ai_[0], ay = ai_[1], az = ai_[2], ah = ai_[3];
            const double bx = bi_[0], by = bi_[1], bz = bi_[2], bh = bi_[3];
            // c_i = a_i . (b_i x n_i), P_i a_i
            const double cc = ax * (by * nz - bz * ny) + ay * (bz * nx - bx * nz) + az * (bx * ny - by * nx);
            const double an = nx * ax + ny * ay + nz * az;
            const double tx = ax - an * nx, ty = ay - an * ny, tz = az - an * nz;
            double zb = 0.0, vcx = 0.0, vcy = 0.0, vcz = 0.0, gq = 0.0, drx = 0.0, dry = 0.0, drz = 0.0;
#pragma unroll
            for (int s = q; s < 6; s += L) {
                const int e = 6 * i + s;
                const int j = M.nbr[e];
                const Cell cj = load_cell(M.cen, j);
                const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
                double aj_[4], bj_[4];
                load4(av, j, aj_);
                load4(bv, j, bj_);
                const double ajx = aj_[0], ajy = aj_[1], ajz = aj_[2], ajh = aj_[3];
                const double bjx = bj_[0], bjy = bj_[1], bjz = bj_[2];
                const double raj = cj.ra;
                zb += w.bx * (bx + bjx) + w.by * (by + bjy) + w.bz * (bz + bjz);
                const double cj_ = ajx * (bjy * cj.z - bjz * cj.y) + ajy * (bjz * cj.x - bjx * cj.z) +
                                   ajz * (bjx * cj.y - bjy * cj.x);
                const double dc = cc * rai - cj_ * raj;
                vcx += w.bx * dc;
                vcy += w.by * dc;
                vcz += w.bz * dc;
                const double ajn = cj.x * ajx + cj.y * ajy + cj.z * ajz;
                const double px = ajx - ajn * cj.x, py = ajy - ajn * cj.y, pz = ajz - ajn * cj.z;
                gq += w.ax * (tx * rai + px * raj) + w.ay * (ty * rai + py * raj) +
                      w.az * (tz * rai + pz * raj);
                const double dh = ah * rai - ajh * raj;
                drx += w.ax * dh;
                dry += w.ay * dh;
                drz += w.az * dh;
            }
            zb = grp_sum<L>(zb);
            vcx = grp_sum<L>(vcx);
            vcy = grp_sum<L>(vcy);
            vcz = grp_sum<L>(vcz);
            gq = grp_sum<L>(gq);
            drx = grp_sum<L>(drx);
            dry = grp_sum<L>(dry);
            drz = grp_sum<L>(drz);
            const double qq = -Ai * gq;
            const double rx = Ai * drx, ry = Ai * dry, rz = Ai * drz;
            // a x n
            const double anx = ay * nz - az * ny, any = az * nx - ax * nz, anz = ax * ny - ay * nx;
            o[0] += cr * (-zb * anx + Ai * vcx - qq * bx - bh * rx);
            o[1] += cr * (-zb * any + Ai * vcy - qq * by - bh * ry);
            o[2] += cr * (-zb * anz + Ai * vcz - qq * bz - bh * rz);
            o[3] += cr * (-(rx * bx + ry * by + rz * bz));
        }
#pragma unroll
        for (int b = q; b < 4; b += L) {
            const int oi = 4 * i + b;
            out[oi] = k.accumulate ? out[oi] + o[b] : o[b];
        }
    }
}

// k_kpairs on grids with chunk tables.  Per chunk, the centres and areas of
// the chunk's cells and their halo are staged once, and each lane forms the
// weights of its edge slots once (edge_weights_short) and keeps them in
// registers over all pairs; per pair, one thread per staged cell loads a_r
// and b_r and stores what the edges take -- c ra, (P a) ra, a_h ra (c =
// a . (b x n), ra = 1/A) and b_vel -- and the chunk's own cells keep a and b.
// Two lanes serve a cell; the pair sums accumulate in registers and the
// chunk's outputs are written once.
constexpr int kKpLdsL = 2;
constexpr int kKpLdsBlock = kChunk * kKpLdsL;

__global__ void __launch_bounds__(kKpLdsBlock, 4) k_kpairs_lds(DevMesh M, KPairArgs k, Batch bt) {
    constexpr int L = kKpLdsL, C = kChunk, S = kChunk + kHaloMax;
    __shared__ double2 gC0[S], gC1[S];                 // centre x, y; centre z, ra
    __shared__ double2 pA[S], pB[S], pC[S], pD[S];     // (c ra, (Pa)_x ra) ((Pa)_y ra, (Pa)_z ra) (a_h ra, b_x) (b_y, b_z)
    __shared__ double2 oA0[C], oA1[C], oB1[C];         // own (a_x, a_y) (a_z, -) (b_z, b_h)
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const int t = threadIdx.x, q = t & (L - 1);
    double *__restrict__ out = member_ptr(k.out, bt.ws, mk);
    const double2 *c2 = reinterpret_cast<const double2 *>(M.cen);
    const Halo &h = M.halo;
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nbx = G / kXcd, xcd = b % kXcd, kk = b / kXcd;
    const ChunkSpan span = xcd_chunks(h.nchunks, xcd);
    const int ck_end = span.end;
    for (int ck = span.first + kk; ck < ck_end; ck += nbx) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        const int h0 = h.hoff[ck], hn = h.hoff[ck + 1] - h0;
        const int li = t / L;
        const bool act = li < cnt;
        const int i = c0 + (act ? li : 0);
        __syncthreads();   // the previous chunk's readers are done
        for (int m = t; m < cnt + hn; m += kKpLdsBlock) {
            const int j = m < cnt ? c0 + m : h.hids[h0 + (m - cnt)];
            const int sl = m < cnt ? m : C + (m - cnt);
            gC0[sl] = c2[2 * (size_t)j];
            gC1[sl] = c2[2 * (size_t)j + 1];
        }
        __syncthreads();
        // this lane's edge weights, kept over the pairs
        EdgeW w[kSlotIter<L>];
        int lj[kSlotIter<L>];
        const double2 I0 = gC0[act ? li : 0], I1 = gC1[act ? li : 0];
        Cell ci;
        ci.x = I0.x;
        ci.y = I0.y;
        ci.z = I1.x;
        ci.ra = I1.y;
#pragma unroll
        for (int s = 0; s < kSlotIter<L>; ++s) {
            const int e = 6 * i + slot_of<L>(q, s);
            lj[s] = h.lnbr[e];
            const double2 J0 = gC0[lj[s]], J1 = gC1[lj[s]];
            Cell cj;
            cj.x = J0.x;
            cj.y = J0.y;
            cj.z = J1.x;
            cj.ra = 0.0;
            w[s] = edge_weights_short(ci, cj, M.cl[e], M.half_r);
        }
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double Ai = 1.0 / ci.ra;
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        for (int pr = 0; pr < k.R; ++pr) {
            const double cr = k.scale * (k.coef ? k.coef[pr] : 1.0);
            if (cr == 0.0) continue;   // the same for every thread of the launch
            const double2 *a2 = reinterpret_cast<const double2 *>(member_ptr(k.a0, bt.ws, mk) + (size_t)pr * k.sa);
            const double2 *b2 = reinterpret_cast<const double2 *>(member_ptr(k.b0, bt.ws, mk) + (size_t)pr * k.sb);
            __syncthreads();   // the previous pair's readers are done
            for (int m = t; m < cnt + hn; m += kKpLdsBlock) {
                const int j = m < cnt ? c0 + m : h.hids[h0 + (m - cnt)];
                const int sl = m < cnt ? m : C + (m - cnt);
                const double2 A0 = a2[2 * (size_t)j], A1 = a2[2 * (size_t)j + 1];
                const double2 B0 = b2[2 * (size_t)j], B1 = b2[2 * (size_t)j + 1];
                const double2 J0 = gC0[sl], J1 = gC1[sl];
                const double cx = J0.x, cy = J0.y, cz = J1.x, ra = J1.y;
                const double ax = A0.x, ay = A0.y, az = A1.x, ah = A1.y;
                const double bx = B0.x, by = B0.y, bz = B1.x;
                const double cc = ax * (by * cz - bz * cy) + ay * (bz * cx - bx * cz) + az * (bx * cy - by * cx);
                const double an = cx * ax + cy * ay + cz * az;
                pA[sl] = make_double2(cc * ra, (ax - an * cx) * ra);
                pB[sl] = make_double2((ay - an * cy) * ra, (az - an * cz) * ra);
                pC[sl] = make_double2(ah * ra, bx);
                pD[sl] = make_double2(by, bz);
                if (m < cnt) {
                    oA0[m] = A0;
                    oA1[m] = A1;
                    oB1[m] = B1;
                }
            }
            __syncthreads();
            if (!act) continue;
            const double2 PA = pA[li], PB = pB[li], PC = pC[li], PD = pD[li];
            const double ci_c = PA.x, tx = PA.y, ty = PB.x, tz = PB.y, hi = PC.x;
            const double bx = PC.y, by = PD.x, bz = PD.y;
            double zb = 0.0, vcx = 0.0, vcy = 0.0, vcz = 0.0, gq = 0.0, drx = 0.0, dry = 0.0, drz = 0.0;
#pragma unroll
            for (int s = 0; s < kSlotIter<L>; ++s) {
                const double2 QA = pA[lj[s]], QB = pB[lj[s]], QC = pC[lj[s]], QD = pD[lj[s]];
                const EdgeW &ww = w[s];
                zb = fma(ww.bz, bz + QD.y, fma(ww.by, by + QD.x, fma(ww.bx, bx + QC.y, zb)));
                const double dc = ci_c - QA.x;
                vcx = fma(ww.bx, dc, vcx);
                vcy = fma(ww.by, dc, vcy);
                vcz = fma(ww.bz, dc, vcz);
                gq = fma(ww.az, tz + QB.y, fma(ww.ay, ty + QB.x, fma(ww.ax, tx + QA.y, gq)));
                const double dh = hi - QC.x;
                drx = fma(ww.ax, dh, drx);
                dry = fma(ww.ay, dh, dry);
                drz = fma(ww.az, dh, drz);
            }
            zb = grp_sum<L>(zb);
            vcx = grp_sum<L>(vcx);
            vcy = grp_sum<L>(vcy);
            vcz = grp_sum<L>(vcz);
            gq = grp_sum<L>(gq);
            drx = grp_sum<L>(drx);
            dry = grp_sum<L>(dry);
            drz = grp_sum<L>(drz);
            const double2 OA0 = oA0[li], OA1 = oA1[li], OB1 = oB1[li];
            const double ax = OA0.x, ay = OA0.y, az = OA1.x, bh = OB1.y;
            const double qq = -Ai * gq;
            const double rx = Ai * drx, ry = Ai * dry, rz = Ai * drz;
            const double anx = ay * nz - az * ny, any = az * nx - ax * nz, anz = ax * ny - ay * nx;
            o[0] += cr * (-zb * anx + Ai * vcx - qq * bx - bh * rx);
            o[1] += cr * (-zb * any + Ai * vcy - qq * by - bh * ry);
            o[2] += cr * (-zb * anz + Ai * vcz - qq * bz - bh * rz);
            o[3] += cr * (-(rx * bx + ry * by + rz * bz));
        }
        if (!act) continue;
#pragma unroll
        for (int kc = 0; kc < kCompIter<L>; ++kc) {
            const int bb = comp_of<L>(q, kc);
            const int oi = 4 * i + bb;
            out[oi] = k.accumulate ? out[oi] + o[bb] : o[bb];
        }
    }
}

// outs[k] (= or +=, bit k of accmask) sum_{r < nv} C[k * ldc + r] v_r,
// v_r = vbase + r * vstride; k < nout <= kMultiOut
__global__ void __launch_bounds__(kBlock) k_lincomb_multi(int n4, MultiArgs a, Batch bt) {
    __shared__ double cf[kMultiOut * kCoefLd];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    for (int e = threadIdx.x; e < a.nout * kCoefLd; e += blockDim.x) cf[e] = a.C[e];
    __syncthreads();
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += gridDim.x * blockDim.x) {
        double acc[kMultiOut];
#pragma unroll
        for (int k = 0; k < kMultiOut; ++k)
            acc[k] = (k < a.nout && a.out[k] && ((a.accmask >> k) & 1)) ? a.out[k][e] : 0.0;
        for (int r = 0; r < a.nv; ++r) {
            const double v = a.vbase[(size_t)r * a.vstride + e];
#pragma unroll
            for (int k = 0; k < kMultiOut; ++k)
                if (k < a.nout) acc[k] += cf[k * kCoefLd + r] * v;
        }
#pragma unroll
        for (int k = 0; k < kMultiOut; ++k)
            if (k < a.nout && a.out[k]) a.out[k][e] = acc[k];
    }
}

// Z_r = sum_{c < nb} z[r * kZLd + c] What_c for r < na (What_c == nullptr: zero)
__global__ void __launch_bounds__(kBlock) k_zgemm(int n4, ZArgs a) {
    __shared__ double cf[kZRows * kZLd];
    for (int e = threadIdx.x; e < a.na * kZLd; e += blockDim.x) cf[e] = a.z[e];
    __syncthreads();
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += gridDim.x * blockDim.x) {
        double x[kZLd];
#pragma unroll
        for (int c = 0; c < kZLd; ++c) x[c] = (c < a.nb && a.w[c]) ? a.w[c][e] : 0.0;
        for (int r = 0; r < a.na; ++r) {
            double z = 0.0;
#pragma unroll
            for (int c = 0; c < kZLd; ++c) z += cf[r * kZLd + c] * x[c];
            a.Z[(size_t)r * a.zstride + e] = z;
        }
    }
}

// ---------------------------------------------------------------------
// Dense exponential of a K x K matrix (K <= kBigMax) by one block, with
// products only, all on the FP64 matrix cores: scaling and squaring around
// the degree-18 Taylor polynomial, evaluated by the Paterson-Stockmeyer
// scheme (powers B^2..B^6, then two Horner steps in B^6: seven products).
// B = A / 2^s with ||B||_1 <= 1.09, where the Taylor remainder
// sum_{k>18} ||B||^k / k! is below 5e-17; then s squarings.  (The forward
// controller keeps the Pade approximant that eq. cost prices; this
// exponential is the adjoint's, which the paper does not have.)
// ---------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

struct BigLds {
    double a[kBigMax * kBigLd];
    double b[kBigMax * kBigLd];
    double red[64];
};

// C = A B (global, row-major, ld K); C may alias A or B.  Both factors are
// staged in LDS first; the product is cut into 16 x 16 output tiles, one wave
// per tile at a time, each K/4 rank-4 steps of v_mfma_f64_16x16x4: lane l
// supplies A(i0 + l%16, k0 + l/16) and B(k0 + l/16, j0 + l%16) and holds
// C(i0 + l/16 + 4 v, j0 + l%16), v < 4.  Entries at or past K enter as
// zeros (read at clamped in-range addresses) and are never written.
__device__ void big_matmul(int K, const double *A, const double *B, double *C, BigLds &L) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int r = e / K, c = e % K;
        L.a[r * kBigLd + c] = A[e];
        L.b[r * kBigLd + c] = B[e];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int nt = (K + 15) >> 4;
    const int li = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < nt * nt; tile += nw) {
        const int i0 = (tile / nt) << 4, j0 = (tile % nt) << 4;
        const int ar = i0 + li, col = j0 + li;
        const int arc = ar < K ? ar : K - 1, colc = col < K ? col : K - 1;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + lk;
            const int kc = k < K ? k : K - 1;
            const double av = L.a[arc * kBigLd + kc];
            const double bv = L.b[kc * kBigLd + colc];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((ar < K && k < K) ? av : 0.0,
                                                       (k < K && col < K) ? bv : 0.0, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = i0 + lk + 4 * v;
            if (row < K && col < K) C[row * K + col] = acc[v];
        }
    }
    __syncthreads();
}

// X = exp(A); work holds 6 K^2 doubles.  Returns the number of squarings.
__device__ int big_expm(int K, const double *A, double *X, double *work, BigLds &L) {
    const int tid = threadIdx.x;
    const int KK = K * K;
    double *P[6];   // P[i] = B^i, i = 1..5 (P[0] unused: I), then B^6 in P[0]'s place
    for (int i = 0; i < 6; ++i) P[i] = work + (size_t)i * KK;
    double *B6 = P[0];
    // 1-norm and the scaling exponent (K <= kBigMax < blockDim: a column per thread)
    double cs = 0.0;
    if (tid < K)
        for (int r = 0; r < K; ++r) cs += fabs(A[r * K + tid]);
    const double nrm = block_max(cs, L.red);
    if (!(nrm <= 1e30)) {   // NaN, inf or absurd: no finite exponential to compute
        for (int e = tid; e < KK; e += blockDim.x) X[e] = __builtin_nan("");
        __syncthreads();
        return -1;
    }
    int s = 0;
    double scale = 1.0;
    while (nrm * scale > 1.09) {
        ++s;
        scale *= 0.5;
    }
    double ck[19];   // 1 / k!
    ck[0] = 1.0;
    for (int k = 1; k <= 18; ++k) ck[k] = ck[k - 1] / k;
    for (int e = tid; e < KK; e += blockDim.x) P[1][e] = A[e] * scale;
    __syncthreads();
    big_matmul(K, P[1], P[1], P[2], L);   // B^2
    big_matmul(K, P[2], P[1], P[3], L);   // B^3
    big_matmul(K, P[2], P[2], P[4], L);   // B^4
    big_matmul(K, P[4], P[1], P[5], L);   // B^5
    big_matmul(K, P[3], P[3], B6, L);     // B^6
    // the degree-5 blocks of the polynomial: Q_j = sum_i ck[6j + i] B^i
    auto q = [&](int j, int e) {
        double v = (e / K == e % K) ? ck[6 * j] : 0.0;
        for (int i = 1; i <= 5; ++i) v += ck[6 * j + i] * P[i][e];
        return v;
    };
    // X = Q_2 + ck[18] B^6; X = Q_1 + B^6 X; X = Q_0 + B^6 X
    for (int e = tid; e < KK; e += blockDim.x) X[e] = q(2, e) + ck[18] * B6[e];
    __syncthreads();
    for (int j = 1; j >= 0; --j) {
        big_matmul(K, B6, X, X, L);
        for (int e = tid; e < KK; e += blockDim.x) X[e] += q(j, e);
        __syncthreads();
    }
    for (int r = 0; r < s; ++r) big_matmul(K, X, X, X, L);
    return s;
}

// Finish the last adjoint IOM2 column, exponentiate tau G (G the corrected
// augmented matrix of the adjoint Krylov space), the error ratio and the
// coefficients of mu_k (row 0) and of the moment increments vbar_j (rows j).
__global__ void __launch_bounds__(1024) k_adj_gexp(PhiCtl *c, AdjGArgs a, double *mat, double *work,
                                                   double *C, AdjOut *out) {
    __shared__ BigLds L;
    const int tid = threadIdx.x;
    if (a.built >= 1 && c->brk == 0 && !c->beta_zero) {
        double tot[1];
        sum_partials<1>(tot, a.nrm_in, a.np, L.red);
        finalize_column(c, a.built, tot[0], tid == 0, L.red);
        __syncthreads();
    }
    const int m = a.m, p = a.p;
    const int brk = c->brk;
    const int bz = c->beta_zero;
    if (bz) {   // mu_{k+1} = 0: nothing to propagate
        for (int e = tid; e < (kPmax + 1) * kCoefLd; e += blockDim.x) C[e] = 0.0;
        if (tid == 0) {
            out->omega = 0.0;
            out->me = 0;
            out->brk = brk;
            out->beta_zero = 1;
            out->status = 0;
        }
        return;
    }
    const int me = (brk > 0 && brk < m) ? brk : m;
    const double h = (brk > 0 && me == brk) ? 0.0 : c->H[me * kMmax + me - 1];
    const int na = me + 1;
    const int K = na + p;
    const double tau = a.tau;
    for (int e = tid; e < K * K; e += blockDim.x) {
        const int r = e / K, q = e % K;
        double v = 0.0;
        if (r < me && q < me) v = tau * c->H[r * kMmax + q];
        else if (r == me && q == me - 1) v = tau * h;
        else if (r == 0 && q == na) v = tau;
        else if (r >= na && r + 1 < K && q == r + 1) v = tau;
        mat[e] = v;
    }
    __syncthreads();
    big_expm(K, mat, mat, work, L);
    const double beta = c->beta;
    // t_k^i / i! for the moment weights
    for (int e = tid; e < (kPmax + 1) * kCoefLd; e += blockDim.x) {
        const int row = e / kCoefLd, r = e % kCoefLd;
        double v = 0.0;
        if (!bz && r < na && row <= p) {
            const double sr = c->sigma[r];
            if (row == 0) {
                v = beta * sr * mat[r * K + 0];
            } else {
                // vbar_j += sum_{l < j} t^(j-1-l)/(j-1-l)! I_l
                const int j = row;
                for (int l = 0; l < j; ++l) {
                    double f = 1.0;
                    for (int i2 = 1; i2 <= j - 1 - l; ++i2) f = f * a.t / i2;
                    v += f * (beta * sr * mat[r * K + na + l]);
                }
            }
        }
        C[e] = v;
    }
    if (tid == 0) {
        const double eps = bz ? 0.0 : beta * fabs(mat[me * K + 0]);
        out->omega = bz ? 0.0 : a.t_out * eps / (tau * a.tol_abs);
        out->me = bz ? 0 : me;
        out->brk = brk;
        out->beta_zero = bz;
        out->status = (beta != beta || out->omega != out->omega) ? XRB_ENAN : 0;
    }
}

// Van Loan: M = int_0^tau a(tau - s) b(s)^T ds is the top-right block of
// exp(tau [[Hbar_mu, e_1 e_last^T], [0, Hhat_y^T]]); the Z coefficients
// fold in beta_mu sigma_r (adjoint raw basis) and beta_y sigma_c (forward
// raw basis) or 1 (the polynomial vectors w_{p-1} .. w_0).
__global__ void __launch_bounds__(1024) k_adj_vanloan(const PhiCtl *c, const PhiCtl *cy,
                                                      AdjVArgs a, double *mat, double *work,
                                                      double *z) {
    __shared__ BigLds L;
    const int tid = threadIdx.x;
    const int me = a.me, my = a.my, p = a.p;
    const int na = me + 1, nb = my + 1 + p, K = na + nb;
    const double tau = a.tau;
    const int brk = c->brk;
    const double h = (brk > 0 && me == brk) ? 0.0 : c->H[me * kMmax + me - 1];
    const int brky = cy->brk;
    const double hy = (my == 0) ? 0.0 : ((brky > 0 && my == brky) ? 0.0 : cy->H[my * kMmax + my - 1]);
    for (int e = tid; e < K * K; e += blockDim.x) {
        const int r = e / K, q = e % K;
        double v = 0.0;
        if (r < na && q < na) {
            if (r < me && q < me) v = tau * c->H[r * kMmax + q];
            else if (r == me && q == me - 1) v = tau * h;
        } else if (r < na) {
            if (r == 0 && q == K - 1) v = tau;
        } else if (q >= na) {
            // (Hhat_y^T)[rr][qq] = Hhat_y[qq][rr]
            const int rr = r - na, qq = q - na;
            double hv = 0.0;
            if (qq < my && rr < my) hv = cy->H[qq * kMmax + rr];
            else if (qq == my && rr == my - 1) hv = hy;
            else if (qq == 0 && rr == my + 1) hv = 1.0;
            else if (qq >= my + 1 && qq + 1 < nb && rr == qq + 1) hv = 1.0;
            v = tau * hv;
        }
        mat[e] = v;
    }
    __syncthreads();
    big_expm(K, mat, mat, work, L);
    const double bmu = c->beta;
    const double by = cy->beta;
    for (int e = tid; e < kZRows * kZLd; e += blockDim.x) {
        const int r = e / kZLd, q = e % kZLd;
        double v = 0.0;
        if (!c->beta_zero && r < na && q < nb) {
            double f;
            if (q <= my) {
                f = (my == 0) ? 0.0 : by * cy->sigma[q];
            } else {
                const int jw = p - (q - my);
                f = ((a.wzero >> jw) & 1) ? 0.0 : 1.0;
            }
            v = bmu * c->sigma[r] * mat[r * K + na + q] * f;
        }
        z[e] = v;
    }
}

template <int L>
void lapT_launch(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s) {
    if (M.halo.nchunks > 0 && L == kLapTLdsL) {
        // the forward LDS Laplacian's grid: at most the chunk count (whole XCDs)
        const int want = M.lap_grid > 0 ? M.lap_grid : 4 * 256;
        const int cap = (M.halo.nchunks + kXcd - 1) / kXcd * kXcd;
        const int grid = want < cap ? want : cap;
        hipLaunchKernelGGL(k_lapT_lds, dim3(grid, b.nm), dim3(kLapTLdsBlock), 0, s, M, psi, out, b);
        return;
    }
    hipLaunchKernelGGL(k_lapT<L>, dim3(cells_grid(M.n, 256, L), b.nm), dim3(256), 0, s, M, psi, out, b);
}

// Returns the number of partials the launch writes per member (0 without an
// epilogue).
template <int L>
int jtv_launch(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    if (M.halo.nchunks > 0 && L == kJtvLdsL && red_parts(M.n) % kXcd == 0) {
        // as the forward LDS product: no more blocks than chunks, except for
        // norm partials, whose consumers sum red_parts(n)
        const int cap = (M.halo.nchunks + kXcd - 1) / kXcd * kXcd;
        const int np = epi == kEpiNorm ? red_parts(M.n) : (cap < red_parts(M.n) ? cap : red_parts(M.n));
        const dim3 grid(np, b.nm), block(kJtvLdsBlock);
        if (epi == kEpiIom2)
            hipLaunchKernelGGL(k_jtv_lds<kEpiIom2>, grid, block, 0, s, M, a, b);
        else if (epi == kEpiNorm)
            hipLaunchKernelGGL(k_jtv_lds<kEpiNorm>, grid, block, 0, s, M, a, b);
        else
            hipLaunchKernelGGL(k_jtv_lds<kEpiNone>, grid, block, 0, s, M, a, b);
        return epi == kEpiNone ? 0 : np;
    }
    if (epi == kEpiNone) {
        hipLaunchKernelGGL((k_jtv<kEpiNone, L>), dim3(cells_grid(M.n, 256, L), b.nm), dim3(256), 0,
                           s, M, a, b);
        return 0;
    }
    const int grid = red_parts(M.n), block = red_block(M.n);
    if (epi == kEpiIom2) {
        hipLaunchKernelGGL((k_jtv<kEpiIom2, L>), dim3(grid, b.nm), dim3(block), 0, s, M, a, b);
    } else {
        const int nb = block < kJtvMaxBlock<kEpiNorm> ? block : kJtvMaxBlock<kEpiNorm>;
        hipLaunchKernelGGL((k_jtv<kEpiNorm, L>), dim3(grid, b.nm), dim3(nb), 0, s, M, a, b);
    }
    return grid;
}

template <int L>
void kpairs_launch(const DevMesh &M, const KPairArgs &k, const Batch &b, hipStream_t s) {
    if (M.halo.nchunks > 0 && L == kKpLdsL) {
        // every chunk once: the chunk count rounded up to whole XCDs
        const int grid = (M.halo.nchunks + kXcd - 1) / kXcd * kXcd;
        hipLaunchKernelGGL(k_kpairs_lds, dim3(grid, b.nm), dim3(kKpLdsBlock), 0, s, M, k, b);
        return;
    }
    hipLaunchKernelGGL(k_kpairs<L>, dim3(cells_grid(M.n, 256, L), b.nm), dim3(256), 0, s, M, k, b);
}

inline int elem_grid(int n4) {
    int g = (n4 + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    return g < 1 ? 1 : g;
}

}  // namespace

void launch_lapT(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s) {
#define XRB_CALL(L) lapT_launch<L>(M, psi, out, b, s)
    XRB_LANES_DISPATCH(XRB_CALL)
#undef XRB_CALL
}

int launch_jtv(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    int np = 0;
#define XRB_CALL(L) np = jtv_launch<L>(M, a, epi, b, s)
    XRB_LANES_DISPATCH(XRB_CALL)
#undef XRB_CALL
    return np;
}

void launch_kpairs(const DevMesh &M, const KPairArgs &k, const Batch &b, hipStream_t s) {
#define XRB_CALL(L) kpairs_launch<L>(M, k, b, s)
    XRB_LANES_DISPATCH(XRB_CALL)
#undef XRB_CALL
}

void launch_lincomb_multi(int n4, const MultiArgs &a, const Batch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb_multi, dim3(elem_grid(n4), b.nm), dim3(kBlock), 0, s, n4, a, b);
}

void launch_zgemm(int n4, const ZArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_zgemm, dim3(elem_grid(n4)), dim3(kBlock), 0, s, n4, a);
}

void launch_adj_gexp(PhiCtl *c, const AdjGArgs &a, double *mat, double *work, double *C,
                     AdjOut *out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_gexp, dim3(1), dim3(1024), 0, s, c, a, mat, work, C, out);
}

void launch_adj_vanloan(const PhiCtl *c, const PhiCtl *cy, const AdjVArgs &a, double *mat,
                        double *work, double *z, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_vanloan, dim3(1), dim3(1024), 0, s, c, cy, a, mat, work, z);
}

}  // namespace xrb
