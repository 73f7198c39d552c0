// Finite-volume stencil kernels of the shallow-water model (Sec. 2):
//   F(u)    eq. sweqsinv with D_f = -nu L^2 (eq. swdis)
//   J(u) x  eqs. dynjs-dynjc, fused with the IOM2 dot products or the w_j
//           recurrence axpys of Alg. 1
//
// Edge-parallel mapping: L consecutive lanes serve one cell (L = 8 on small
// grids, where the extra memory-level parallelism pays; fewer on large
// ones, where the per-cell work repeated in every lane of the group would
// cost more than it hides).  Each lane gathers its neighbours, forms their
// edge terms, and a fixed DPP butterfly over the L lanes sums them (bitwise
// identical in all L).  The two-ring dissipation stencil L(L x) takes L x
// from a preceding one-ring pass (launch_lap4), or, in small eight-lane
// launches, forms it in the product kernel with the same rounding.
#include "column.h"
#include "reduce.h"
#include "stencil_common.h"
#include "xrb_internal.h"

namespace xrb {

int stencil_lanes(int n) { return n > 16384 ? 2 : 8; }

// The product forms L x itself (eight lanes per cell) for launches over few
// cells in all, where the saved launch and round trip pay; large grids and
// ensembles keep the separate k_lap4 pass (the extra gathers cost more
// there).  Both forms give the same bits.
bool jv_fuses_lap(const DevMesh &M, int nm) { return M.lanes == 8 && (long)nm * M.n <= 200000L; }

// Lanes per cell of a forward stencil launch over nm members: few cells in
// all take M.lanes (more memory-level parallelism per cell, for latency),
// many take M.lanes_batch (fewer repeated per-cell instructions, for
// throughput).  Two and eight lanes give the same bits on grids without
// chunk tables (lanes_pair_bitwise).
int launch_lanes(const DevMesh &M, int nm) {
    return (long)nm * M.n > 200000L ? M.lanes_batch : M.lanes;
}

// Whether single-state launches with a lanes and batched ones with b give
// the same bits: the same count, or two and eight on grids whose reducing
// products reduce per-cell terms in fixed order and have no chunk tables.
bool lanes_pair_bitwise(const DevMesh &M, int a, int b) {
    if (a == b) return true;
    const bool two_eight = (a == 2 || a == 8) && (b == 2 || b == 8);
    // with chunk tables two lanes take the LDS-staged product, whose rounding
    // is its own
    return two_eight && stc::red_cells(M.n) <= stc::kCellRedMax && M.halo.nchunks == 0;
}

namespace {

using namespace stc;

// Every stencil serves a cell with L consecutive lanes (L = 1, 2, 4, 8):
// lane q takes the neighbour slots slot_of<L>(q, k) and writes the output
// components comp_of<L>(q, k); the lanes' edge sums, accumulated with
// acc_add, are combined by grp_sum<L>, so two and eight lanes give the same
// bits.  Pentagon slot 5 points at the cell itself with zero weights.

template <int L>
__global__ void __launch_bounds__(256) k_lap4(DevMesh M, const double *__restrict__ psi,
                                              double *__restrict__ out, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    psi = member_ptr(psi, bt.ws, mk);
    out = member_ptr(out, bt.ws, mk);
    const int n = M.n;
    const int q = threadIdx.x & (L - 1);
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        double pi[4];
        load4(psi, i, pi);
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int s = slot_of<L>(q, k);
            if (s < 0) continue;
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            const double c = M.cl[e];
            double pj[4];
            load4(psi, j, pj);
#pragma unroll
            for (int b = 0; b < 4; ++b) a[b] = acc_add(a[b], c * (pj[b] - pi[b]));
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) a[b] = grp_sum<L>(a[b]);
#pragma unroll
        for (int k = 0; k < kCompIter<L>; ++k) {
            const int b = comp_of<L>(q, k);
            if (b >= 0) out[4 * i + b] = a[b];
        }
    }
}

// L x of large grids with the chunk's cells and their one-ring halo staged
// in LDS (the chunk tables of k_jv_lds): the per-cell arithmetic, lane
// placement and sums of k_lap4<kJvLdsL>, so the same bits.  Any grid that
// is a multiple of the XCD count.
constexpr int kLapLdsL = 2;
constexpr int kLapLdsBlock = kChunk * kLapLdsL;

__global__ void __launch_bounds__(kLapLdsBlock) k_lap4_lds(DevMesh M, const double *__restrict__ psi,
                                                           double *__restrict__ out, Batch bt) {
    constexpr int L = kLapLdsL, C = kChunk, HM = kHaloMax;
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
        for (int k = t; k < 2 * cnt; k += kLapLdsBlock) sx[k] = x2[2 * (size_t)c0 + k];
        for (int k = t; k < 2 * hn; k += kLapLdsBlock)
            sx[2 * C + k] = x2[2 * (size_t)h.hids[h0 + (k >> 1)] + (k & 1)];
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
            for (int bb = 0; bb < 4; ++bb) acc[bb] = acc_add(acc[bb], c * (pj[bb] - pi[bb]));
        }
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[bb] = grp_sum<L>(acc[bb]);
#pragma unroll
        for (int k = 0; k < kCompIter<L>; ++k) out[4 * i + comp_of<L>(q, k)] = acc[comp_of<L>(q, k)];
    }
}

// The chunked IOM2 update of column j on grids with chunk tables (512
// threads per block, chunks XCD-major).  Every block first takes the update's
// prologue (the column's dots and norm from the partials, its scale and H
// entries: iom2_coefficients).  Per chunk, thread t forms pair t of the
// chunk's cells, t < 2 cnt, of R_{j+1} = sj w - cj R_j - cm R_{j-1}
// (iom2_pair) and adds x.x^2 + x.y^2 to its share of ||R_{j+1}||^2.  With
// per_chunk the shares are summed by block_sum_all after every chunk and
// stored at the chunk's index (any grid gives the same bits); without, once
// per block at the block's index (the grid must be the same).  The two
// kernels below do exactly that, so they give the same bits.
constexpr int kUpdLapL = 2;
constexpr int kUpdLapBlock = kChunk * kUpdLapL;

// R_{j+1} over w in place, with the column-norm partials.
__global__ void __launch_bounds__(kUpdLapBlock) k_iom2_update_lds(DevMesh M, int j, double *w,
                                                                 const double *rj, const double *rjm1,
                                                                 PhiCtl *ctl0, const double *nrm_in,
                                                                 int np_nrm, const double *dot_in,
                                                                 int np_dot, double *nrm_out,
                                                                 int per_chunk, Batch bt) {
    constexpr int C = kChunk, NW = kUpdLapBlock / 64;
    // per-chunk mode: the wave sums of the block's chunks (at most
    // ceil(kNrmRegion / kXcd) chunks per block), combined once at the end in
    // block_sum_all's order
    __shared__ double wsum[(kNrmRegion / kXcd) * NW];
    __shared__ double pro[16 * 4];
    __shared__ double lds[16];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    double2 *w2 = reinterpret_cast<double2 *>(member_ptr(w, bt.ws, mk));
    const double2 *r2 = reinterpret_cast<const double2 *>(member_ptr(rj, bt.ws, mk));
    const double2 *m2 = reinterpret_cast<const double2 *>(member_ptr(j > 0 ? rjm1 : rj, bt.ws, mk));
    double *parts = nrm_out + (size_t)mk * kPartStride;
    const Halo &h = M.halo;
    const int n = M.n;
    const int t = threadIdx.x;
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nbx = G / kXcd, xcd = b % kXcd, kk = b / kXcd;
    const ChunkSpan span = xcd_chunks(h.nchunks, xcd);
    const int ck_end = span.end;
    const double2 z2 = make_double2(0.0, 0.0);
    double2 pw = z2, pr = z2, pm = z2;
    auto fetch = [&](int ck) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        const bool in = t < 2 * cnt;
        const size_t e = 2 * (size_t)c0 + (in ? t : 0);
        pw = in ? w2[e] : z2;
        pr = in ? r2[e] : z2;
        pm = (in && j > 0) ? m2[e] : z2;
    };
    const int ck0 = span.first + kk;
    if (ck0 < ck_end) fetch(ck0);
    PhiCtl *ctl = ctl_member(ctl0, mk);
    // a new basis (j = 0) starts fresh; later columns stop after a breakdown
    if (j > 0 && (ctl->brk != 0 || ctl->beta_zero)) return;
    const IomCoef kc = iom2_coefficients(ctl, j, mk, nrm_in, np_nrm, dot_in, np_dot, pro);
    if (kc.stop) return;
    double r = 0.0;
    int nck = 0;   // chunks this block took
    for (int ck = ck0; ck < ck_end; ck += nbx, ++nck) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        if (ck != ck0) fetch(ck);
        if (t < 2 * cnt) {
            const double2 x = iom2_pair(kc, j, pw, pr, pm);
            w2[2 * (size_t)c0 + t] = x;
            r += fma(x.y, x.y, x.x * x.x);
        }
        if (per_chunk) {
            const double sw = wave_sum(r);   // valid in lane 0
            if ((t & 63) == 0) wsum[nck * NW + (t >> 6)] = sw;
            r = 0.0;
        }
    }
    if (per_chunk) {
        // chunk c's total as block_sum_all forms it: the wave sums in wave order
        __syncthreads();
        if (t < nck) {
            double tot = 0.0;
#pragma unroll
            for (int v = 0; v < NW; ++v) tot += wsum[t * NW + v];
            parts[ck0 + t * nbx] = tot;
        }
    } else {
        double vv[1] = {r};
        block_sum_all<1>(vv, lds);
        if (t == 0) parts[blockIdx.x] = vv[0];
    }
}

// The same update fused with the Laplacian pass of column j+1: per chunk, the
// pairs of R_{j+1} are formed for the chunk's cells and its one-ring halo into
// LDS (the same instructions for both, so a halo copy has the bits its owner
// writes; the own pairs are pair t of k_iom2_update_lds), the own ones go to
// rn with the chunk's norm partial, and L R_{j+1} of the chunk's cells goes
// to lapn with the arithmetic of k_lap4_lds.  w is the product's output in a
// buffer of its own (rn is written while other blocks still read w).
__global__ void __launch_bounds__(kUpdLapBlock) k_upd_lap_lds(DevMesh M, int j, const double *w,
                                                             const double *rj, const double *rjm1,
                                                             double *rn, double *lapn, PhiCtl *ctl0,
                                                             const double *nrm_in, int np_nrm,
                                                             const double *dot_in, int np_dot,
                                                             double *nrm_out, int per_chunk, Batch bt) {
    constexpr int L = kUpdLapL, C = kChunk, HM = kHaloMax;
    // a chunk and its halo hold at most 2 (C + HM) pairs: two per thread, and
    // the own pairs (2 C) all come first
    static_assert(2 * (C + HM) <= 2 * kUpdLapBlock && 2 * C <= kUpdLapBlock, "staged pairs per thread");
    __shared__ double2 sx[(C + HM) * 2];
    __shared__ double pro[16 * 4];
    __shared__ double lds[16];
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const double2 *w2 = reinterpret_cast<const double2 *>(member_ptr(w, bt.ws, mk));
    const double2 *r2 = reinterpret_cast<const double2 *>(member_ptr(rj, bt.ws, mk));
    const double2 *m2 = reinterpret_cast<const double2 *>(member_ptr(j > 0 ? rjm1 : rj, bt.ws, mk));
    double2 *n2 = reinterpret_cast<double2 *>(member_ptr(rn, bt.ws, mk));
    double *__restrict__ lout = member_ptr(lapn, bt.ws, mk);
    double *parts = nrm_out + (size_t)mk * kPartStride;
    const Halo &h = M.halo;
    const int n = M.n;
    const int t = threadIdx.x, q = t & (L - 1);
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int nbx = G / kXcd, xcd = b % kXcd, kk = b / kXcd;
    const ChunkSpan span = xcd_chunks(h.nchunks, xcd);
    const int ck_end = span.end;
    const double2 z2 = make_double2(0.0, 0.0);
    // the thread's staged pairs of a chunk: pair k = t + u kUpdLapBlock, u < 2
    double2 pw[2], pr[2], pm[2];
    auto fetch = [&](int ck) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        const int h0 = h.hoff[ck], hn = h.hoff[ck + 1] - h0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = t + u * kUpdLapBlock;
            const int m = k >> 1;
            const bool in = k < 2 * (cnt + hn);
            const int cell = !in ? 0 : (m < cnt ? c0 + m : h.hids[h0 + (m - cnt)]);
            const size_t e = 2 * (size_t)cell + (k & 1);
            pw[u] = in ? w2[e] : z2;
            pr[u] = in ? r2[e] : z2;
            pm[u] = (in && j > 0) ? m2[e] : z2;
        }
    };
    // (requesting the first chunk before the prologue, as the batched update
    // does, measured slower here: more registers, no gain in latency)
    PhiCtl *ctl = ctl_member(ctl0, mk);
    // a new basis (j = 0) starts fresh; later columns stop after a breakdown
    if (j > 0 && (ctl->brk != 0 || ctl->beta_zero)) return;
    const IomCoef kc = iom2_coefficients(ctl, j, mk, nrm_in, np_nrm, dot_in, np_dot, pro);
    if (kc.stop) return;
    double r = 0.0;
    for (int ck = span.first + kk; ck < ck_end; ck += nbx) {
        const int c0 = ck * C, cnt = min(C, n - c0);
        const int hn = h.hoff[ck + 1] - h.hoff[ck];
        fetch(ck);
        __syncthreads();   // the previous chunk's readers are done
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int k = t + u * kUpdLapBlock;
            if (k >= 2 * (cnt + hn)) continue;
            const int m = k >> 1;
            const bool own = m < cnt;
            const double2 x = iom2_pair(kc, j, pw[u], pr[u], pm[u]);
            sx[(own ? 2 * m : 2 * (C + m - cnt)) + (k & 1)] = x;
            if (own) {   // only u = 0: one pair per chunk, as in k_iom2_update_lds
                n2[2 * (size_t)c0 + k] = x;
                r += fma(x.y, x.y, x.x * x.x);
            }
        }
        if (per_chunk) {
            double vv[1] = {r};
            block_sum_all<1>(vv, lds);
            if (t == 0) parts[ck] = vv[0];
            r = 0.0;
        }
        __syncthreads();   // publishes sx
        const int li = t / L;
        if (li >= cnt) continue;
        const int i = c0 + li;
        const double2 a0 = sx[2 * li], a1 = sx[2 * li + 1];
        const double pi[4] = {a0.x, a0.y, a1.x, a1.y};
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < kSlotIter<L>; ++s) {
            const int e = 6 * i + slot_of<L>(q, s);
            const int lj = h.lnbr[e];
            const double c = M.cl[e];
            const double2 b0 = sx[2 * lj], b1 = sx[2 * lj + 1];
            const double pj[4] = {b0.x, b0.y, b1.x, b1.y};
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) acc[bb] = acc_add(acc[bb], c * (pj[bb] - pi[bb]));
        }
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) acc[bb] = grp_sum<L>(acc[bb]);
#pragma unroll
        for (int s = 0; s < kCompIter<L>; ++s) lout[4 * i + comp_of<L>(q, s)] = acc[comp_of<L>(q, s)];
    }
    if (!per_chunk) {
        double vv[1] = {r};
        block_sum_all<1>(vv, lds);
        if (t == 0) parts[blockIdx.x] = vv[0];
    }
}

template <int L>
__global__ void __launch_bounds__(256) k_linearize(DevMesh M, const double *__restrict__ u,
                                                   double *__restrict__ eta,
                                                   double *__restrict__ rec, Batch bt) {
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    u = member_ptr(u, bt.ws, mk);
    eta = member_ptr(eta, bt.ws, mk);
    rec = member_ptr(rec, bt.ws, mk);
    const int n = M.n;
    const int q = threadIdx.x & (L - 1);
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        const Cell ci = load_cell(M.cen, i);
        double ui[4];
        load4(u, i, ui);
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int s = slot_of<L>(q, k);
            if (s < 0) continue;
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            const Cell cj = load_cell(M.cen, j);
            const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
            double uj[4];
            load4(u, j, uj);
            z = acc_add(z, w.bx * (ui[0] + uj[0]) + w.by * (ui[1] + uj[1]) + w.bz * (ui[2] + uj[2]));
        }
        z = grp_sum<L>(z);
        const double et = z + M.two_omega * ci.z;
        if (q == 0) eta[i] = et;
        if (rec) {
            // record (u_x, u_y, u_z, h, x, y, z, eta): two 16-byte stores per lane
            // pair position, spread over the group's lanes
            const double v[8] = {ui[0], ui[1], ui[2], ui[3], ci.x, ci.y, ci.z, et};
            double2 *r2 = reinterpret_cast<double2 *>(rec) + 4 * (size_t)i;
#pragma unroll
            for (int k = q; k < 4; k += L) r2[k] = make_double2(v[2 * k], v[2 * k + 1]);
        }
    }
}

template <int L>
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
    const int q = threadIdx.x & (L - 1);
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        double ui[4], lui[4];
        load4(u, i, ui);
        load4(lu, i, lui);
        const double ux = ui[0], uy = ui[1], uz = ui[2], h = ui[3];
        const Cell ci = load_cell(M.cen, i);
        // E = |u|^2 / 2 + g (h + h_s)
        const double Ei = 0.5 * (ux * ux + uy * uy + uz * uz) + g * (M.hs ? h + M.hs[i] : h);
        double gx = 0.0, gy0 = 0.0, gz0 = 0.0, dv = 0.0, zt = 0.0;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            // edge terms without contraction: h u_i is loop-invariant, so an
            // unrolled two-lane loop (one product, three uses) and a one-edge
            // eight-lane body (one use) would fuse it differently
#pragma clang fp contract(off)
            const int s = slot_of<L>(q, k);
            if (s < 0) continue;
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            double uj[4], luj[4];
            load4(u, j, uj);
            load4(lu, j, luj);
            const double vx = uj[0], vy = uj[1], vz = uj[2], hj = uj[3];
            const Cell cj = load_cell(M.cen, j);
            const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
            const double c = M.cl[e];
            const double Ej = 0.5 * (vx * vx + vy * vy + vz * vz) + g * (M.hs ? hj + M.hs[j] : hj);
            const double dE = Ej - Ei;
            gx = acc_add(gx, w.ax * dE);
            gy0 = acc_add(gy0, w.ay * dE);
            gz0 = acc_add(gz0, w.az * dE);
            dv = acc_add(dv, w.ax * (h * ux + hj * vx) + w.ay * (h * uy + hj * vy) +
                                 w.az * (h * uz + hj * vz));
            zt = acc_add(zt, w.bx * (ux + vx) + w.by * (uy + vy) + w.bz * (uz + vz));
#pragma unroll
            for (int b = 0; b < 4; ++b) d[b] = acc_add(d[b], c * (luj[b] - lui[b]));
        }
        gx = grp_sum<L>(gx);
        gy0 = grp_sum<L>(gy0);
        gz0 = grp_sum<L>(gz0);
        dv = grp_sum<L>(dv);
        zt = grp_sum<L>(zt);
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = grp_sum<L>(d[b]);
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double gr = nx * gx + ny * gy0 + nz * gz0;       // tangent projection of grad E
        const double Gx = gx - gr * nx, Gy = gy0 - gr * ny, Gz = gz0 - gr * nz;
        const double eta = zt + M.two_omega * ci.z;
        const double px = ny * uz - nz * uy, py = nz * ux - nx * uz, pz = nx * uy - ny * ux;
        const double nu = M.nu;
        double o[4];
        o[0] = -eta * px - Gx - nu * d[0];
        o[1] = -eta * py - Gy - nu * d[1];
        o[2] = -eta * pz - Gz - nu * d[2];
        o[3] = -dv - nu * d[3];
#pragma unroll
        for (int k = 0; k < kCompIter<L>; ++k) {
            const int b = comp_of<L>(q, k);
            if (b >= 0) f[4 * i + b] = o[b];
        }
    }
}

// out = dt*J(u) x + sum_k c_k v_k, with an optional reduction epilogue
// (IOM2: raw dot partials; recurrence: norm partials).
// FL (eight lanes per cell only): the two-ring dissipation term takes L x
// from inside the kernel instead of from a preceding k_lap4 pass -- one
// launch and one vector round trip less per product, for more gathers per
// lane.  Each lane forms L x at its neighbour j over j's ring with the sum
// tree k_lap4 applies, ((t0 + t2) + t4) + ((t1 + t3) + t5), products rounded
// on their own; L x at i is the group sum of the lanes' own-edge terms.  The result is therefore bit-identical to the
// two-pass form, and the launcher may choose either per call.
// Threads per block at most: the plain product and the norm variant 256
// (the register budget that bound allows keeps them free of spills), the
// IOM2 variant 1024.
template <int EPI>
constexpr int kJvMaxBlock = EPI == kEpiIom2 ? 1024 : 256;

template <int EPI, int L, bool FL, bool CR>
__global__ void __launch_bounds__(kJvMaxBlock<EPI>) k_jv(DevMesh M, JvArgs a, Batch bt) {
    __shared__ double lds[64];
    __shared__ double cterm[2 * kCellRedMax];   // per-cell reduction terms
    const int mk = blockIdx.y;
    if (!member_active(bt.pred, mk)) return;
    const int n = M.n;
    const double g = M.g, nu = M.nu;
    const double sc = bt.dtk ? bt.dtk[mk] : a.dt;
    // small grids reduce per-cell terms (fixed order, any block size);
    // large ones accumulate per lane (block size fixed by n)
    // CR: the launch's chunks hold at most kCellRedMax cells (the launcher
    // decides from red_cells(n)); such launches run one pass per block, where
    // requesting the epilogue's own-cell operands with the gathers pays, while
    // the multi-pass launches of large grids keep their registers for the loop
    constexpr bool cellred = EPI != kEpiNone && CR;
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
    double r0 = 0.0, r1 = 0.0;   // this lane's reduction partials
    // per-cell reduction needs each block's cells contiguous; the per-lane
    // accumulation of large grids sweeps each XCD's cells window by window
    const CellRange r_init = cellred ? block_cells<L>(n) : block_cells_swept<L>(n);
    for (CellRange r = r_init; r.i < r.end; r.i += r.step) {
        const int i = r.i;
        double ui[4], xi[4], lxo[4] = {0.0, 0.0, 0.0, 0.0};
        load4(u, i, ui);
        load4(x, i, xi);
        if (!FL) load4(lx, i, lxo);
        const double ux = ui[0], uy = ui[1], uz = ui[2], uh = ui[3];
        const double xx = xi[0], xy = xi[1], xz = xi[2], xh = xi[3];
        const Cell ci = load_cell(M.cen, i);
        // one-pass launches request the cell's own epilogue operands with
        // the gathers, not after them
        double eta = 0.0;
        double pm[kCompIter<L>];
        if constexpr (cellred) {
            eta = etak[i];
#pragma unroll
            for (int kc = 0; kc < kCompIter<L>; ++kc) {
                const int b = comp_of<L>(q, kc);
                pm[kc] = (EPI == kEpiIom2 && rjm1 && b >= 0) ? rjm1[4 * i + b] : 0.0;
            }
        }
        const double si = ux * xx + uy * xy + uz * xz + g * xh;       // u.x_vel + g x_h
        const double fx = uh * xx + xh * ux, fy = uh * xy + xh * uy, fz = uh * xz + xh * uz;
        double gx = 0.0, gy0 = 0.0, gz0 = 0.0, dv = 0.0, zt = 0.0;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
        double lxi[4] = {0.0, 0.0, 0.0, 0.0};   // FL: this lane's edge term of L x at i
        double lxj[4] = {0.0, 0.0, 0.0, 0.0};   // FL: L x at this lane's neighbour
        double cl_s = 0.0;                      // FL: this lane's c (0 without an edge)
        const double xs_i[4] = {xx, xy, xz, xh};
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int s = slot_of<L>(q, k);
            if (s < 0) continue;
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            double xj[4], uj[4];
            load4(x, j, xj);
            load4(u, j, uj);
            const double vx = xj[0], vy = xj[1], vz = xj[2], vh = xj[3];
            const double wx = uj[0], wy = uj[1], wz = uj[2], wh = uj[3];
            const Cell cj = load_cell(M.cen, j);
            const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
            const double c = M.cl[e];
            const double sj = wx * vx + wy * vy + wz * vz + g * vh;
            const double ds = sj - si;
            gx = acc_add(gx, w.ax * ds);
            gy0 = acc_add(gy0, w.ay * ds);
            gz0 = acc_add(gz0, w.az * ds);
            dv = acc_add(dv, w.ax * (fx + (wh * vx + vh * wx)) + w.ay * (fy + (wh * vy + vh * wy)) +
                                 w.az * (fz + (wh * vz + vh * wz)));
            zt = acc_add(zt, w.bx * (xx + vx) + w.by * (xy + vy) + w.bz * (xz + vz));
            if (FL) {
                // no contraction: every product is rounded on its own, as the
                // single-term lane sums of the two-pass form are
#pragma clang fp contract(off)
                const double xs_j[4] = {vx, vy, vz, vh};
                double t[6][4];
#pragma unroll
                for (int tt = 0; tt < 6; ++tt) {
                    const int ej = 6 * j + tt;
                    const int kk = M.nbr[ej];
                    const double cj = M.cl[ej];
                    double xk[4];
                    load4(x, kk, xk);
#pragma unroll
                    for (int b = 0; b < 4; ++b) t[tt][b] = cj * (xk[b] - xs_j[b]);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    lxj[b] = ((t[0][b] + t[2][b]) + t[4][b]) + ((t[1][b] + t[3][b]) + t[5][b]);
                    lxi[b] = c * (xs_j[b] - xs_i[b]);
                }
                cl_s = c;
            } else {
                double lxj_[4];
                load4(lx, j, lxj_);
#pragma unroll
                for (int b = 0; b < 4; ++b) d[b] = acc_add(d[b], c * (lxj_[b] - lxo[b]));
            }
        }
        if (FL) {
            // the two-pass form's d = group sum of c_s (L x_j - L x_i)
#pragma clang fp contract(off)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double li = grp_sum<L>(lxi[b]);
                const double ts = cl_s * (lxj[b] - li);
                d[b] = grp_sum<L>(ts);
            }
        }
        gx = grp_sum<L>(gx);
        gy0 = grp_sum<L>(gy0);
        gz0 = grp_sum<L>(gz0);
        dv = grp_sum<L>(dv);
        zt = grp_sum<L>(zt);
        if (!FL) {
#pragma unroll
            for (int b = 0; b < 4; ++b) d[b] = grp_sum<L>(d[b]);
        }
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double gr = nx * gx + ny * gy0 + nz * gz0;
        const double Gx = gx - gr * nx, Gy = gy0 - gr * ny, Gz = gz0 - gr * nz;
        if constexpr (!cellred) eta = etak[i];
        // J_v x: -(V.x) (n x u);  J_r x: -eta (n x x) - nu L^2 x;
        // J_m x: -G(u.x + g x_h), -D(h x + x_h u)
        const double pux = ny * uz - nz * uy, puy = nz * ux - nx * uz, puz = nx * uy - ny * ux;
        const double pxx = ny * xz - nz * xy, pxy = nz * xx - nx * xz, pxz = nx * xy - ny * xx;
        double o[4];
        o[0] = sc * (-zt * pux - eta * pxx - Gx - nu * d[0]);
        o[1] = sc * (-zt * puy - eta * pxy - Gy - nu * d[1]);
        o[2] = sc * (-zt * puz - eta * pxz - Gz - nu * d[2]);
        o[3] = sc * (-dv - nu * d[3]);
        const double xs[4] = {xx, xy, xz, xh};
        double c0 = 0.0, c1 = 0.0;   // this lane's terms of the cell
#pragma unroll
        for (int kc = 0; kc < kCompIter<L>; ++kc) {
            const int b = comp_of<L>(q, kc);
            if (b < 0) continue;
            const int oi = 4 * i + b;
            double ob = o[b];
#pragma unroll
            for (int k = 0; k < kPmax; ++k)
                if (k < a.naxpy) ob += cax[k] * axv[k][oi];
            outk[oi] = ob;
            if (EPI == kEpiIom2) {
                c0 = acc_add(c0, ob * xs[b]);
                if (rjm1) c1 = acc_add(c1, ob * (cellred ? pm[kc] : rjm1[oi]));
            } else if (EPI == kEpiNorm) {
                c0 = acc_add(c0, ob * ob);
            }
        }
        if (EPI != kEpiNone) {
            if (cellred) {
                c0 = grp_sum<L>(c0);
                if (EPI == kEpiIom2) c1 = grp_sum<L>(c1);
                if (q == 0) {
                    cterm[2 * (i - r.first)] = c0;
                    cterm[2 * (i - r.first) + 1] = c1;
                }
            } else {
                r0 += c0;
                r1 += c1;
            }
        }
    }
    if (EPI == kEpiNone) return;
    double *parts = (EPI == kEpiIom2 ? a.dot_out : a.nrm_out) + (size_t)mk * kPartStride;
    constexpr int NV = EPI == kEpiIom2 ? 2 : 1;
    if (cellred) {
        // cell terms summed by the first wave in cell order
        __syncthreads();
        if (threadIdx.x < 64) {
            const int cnt = r_init.end - r_init.first;
            double v[2] = {0.0, 0.0};
            for (int c = (int)threadIdx.x; c < cnt; c += 64) {
                v[0] += cterm[2 * c];
                v[1] += cterm[2 * c + 1];
            }
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
            if (threadIdx.x == 0)
#pragma unroll
                for (int k = 0; k < NV; ++k) parts[blockIdx.x * NV + k] = v[k];
        }
        return;
    }
    double v[2] = {r0, r1};
    block_sum_all<2>(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) parts[blockIdx.x * NV + k] = v[k];
}

// The product of large grids with its neighbours staged in LDS.  Block b
// takes chunks of kChunk consecutive cells (XCD-major: the blocks on XCD x
// sweep that die's contiguous share of the chunks, xcd_chunks, together,
// window by window).  For each
// chunk, one thread per cell of the chunk and of its one-ring halo loads the
// cell's x, L x and linearisation record (u, centre, eta) and stores in LDS
// what its edges need: s = u . x_vel + g x_h, the flux F = h x_vel + x_h u
// and P = x_vel x c (c the unit centre), all formed once per cell instead of
// once per edge, the centre and L x -- 14 doubles; the chunk's own cells
// also keep u, eta and x.  Every edge term then reads its neighbour from LDS
// through the chunk's 16-bit local ids, with alpha and beta formed from c
// and the chord by the NT-term series (edge_ab_short).  The circulation term
// beta (c_i x c_j) . (x_i + x_j) is taken as beta (P_i . c_j - P_j . c_i)
// (the two scalar triple products), which needs no cross product per edge.
// Two lanes serve a cell (kJvLdsL), with the lane
// placement and sums of k_jv<EPI, 2>; the rounding differs from the gather
// kernels (weights from the series, no stored alpha), so a grid with chunk
// tables keeps this kernel for all its two-lane products.  Reductions:
// per-lane partials over the block's chunks, then one block sum
// (red_parts(n) blocks).
constexpr int kJvLdsL = 2;
constexpr int kJvLdsBlock = kChunk * kJvLdsL;

template <int EPI, int NT>
__global__ void __launch_bounds__(kJvLdsBlock, 4) k_jv_lds(DevMesh M, JvArgs a, Batch bt) {
    constexpr int L = kJvLdsL, C = kChunk, S = kChunk + kHaloMax;
    // staged cells (chunk, then halo): (s, F_x) (F_y, F_z) (P_x, P_y) (P_z, centre_x)
    // (centre_y, centre_z) (Lx_0, Lx_1) (Lx_2, Lx_3); the chunk's own cells:
    // (u_x, u_y) (u_z, x_z) (eta, x_h) (x_x, x_y)
    __shared__ double2 nA[S], nB[S], nC[S], nD[S], nE[S], nL0[S], nL1[S];
    __shared__ double2 oU0[C], oU1[C], oE[C], oX[C];
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
    const double2 *l2 = reinterpret_cast<const double2 *>(member_ptr(a.lx, bt.ws, mk));
    const double2 *r2 = reinterpret_cast<const double2 *>(member_ptr(a.rec, bt.ws, mk));
    double *__restrict__ outk = member_ptr(a.out, bt.ws, mk);
    // column 0 has no R_{-1}: its second dot runs against x and is ignored by
    // the update (h_{-1,0} is not formed), which saves a branch per cell
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
        for (int m = t; m < cnt + hn; m += kJvLdsBlock) {
            const bool own = m < cnt;
            const int j = own ? c0 + m : h.hids[h0 + (m - cnt)];
            const int sl = own ? m : C + (m - cnt);
            const double2 v0 = x2[2 * (size_t)j], v1 = x2[2 * (size_t)j + 1];
            const double2 w0 = r2[4 * (size_t)j], w1 = r2[4 * (size_t)j + 1];
            const double2 w2 = r2[4 * (size_t)j + 2], w3 = r2[4 * (size_t)j + 3];
            nL0[sl] = l2[2 * (size_t)j];
            nL1[sl] = l2[2 * (size_t)j + 1];
            const double vx = v0.x, vy = v0.y, vz = v1.x, vh = v1.y;
            const double wx = w0.x, wy = w0.y, wz = w1.x, wh = w1.y;
            const double cx = w2.x, cy = w2.y, cz = w3.x;
            nA[sl] = make_double2(wx * vx + wy * vy + wz * vz + g * vh, wh * vx + vh * wx);
            nB[sl] = make_double2(wh * vy + vh * wy, wh * vz + vh * wz);
            nC[sl] = make_double2(vy * cz - vz * cy, vz * cx - vx * cz);
            nD[sl] = make_double2(vx * cy - vy * cx, cx);
            nE[sl] = make_double2(cy, cz);
            if (own) {
                oU0[m] = w0;
                oU1[m] = make_double2(wz, vz);
                oE[m] = make_double2(w3.y, vh);
                oX[m] = v0;
            }
        }
        __syncthreads();
        const int li = t / L;
        if (li >= cnt) continue;
        const int i = c0 + li;
        const double2 A0 = nA[li], B0 = nB[li], C0 = nC[li], D0 = nD[li], E0 = nE[li];
        const double2 s0 = nL0[li], s1 = nL1[li];
        Cell ci;
        ci.x = D0.y;
        ci.y = E0.x;
        ci.z = E0.y;
        ci.ra = 0.0;
        const double pix = C0.x, piy = C0.y, piz = D0.x;
        const double lxo[4] = {s0.x, s0.y, s1.x, s1.y};
        const double si = A0.x, fx = A0.y, fy = B0.x, fz = B0.y;
        double gx = 0.0, gy0 = 0.0, gz0 = 0.0, dv = 0.0, zt = 0.0;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int e = 6 * i + slot_of<L>(q, k);
            const int lj = h.lnbr[e];
            const double c = M.cl[e];
            const double2 Aj = nA[lj], Bj = nB[lj], Cj = nC[lj], Dj = nD[lj], Ej = nE[lj];
            const double2 e0 = nL0[lj], e1 = nL1[lj];
            Cell cj;
            cj.x = Dj.y;
            cj.y = Ej.x;
            cj.z = Ej.y;
            cj.ra = 0.0;
            double al, be, dx, dy, dz;
            edge_ab_short<NT>(ci, cj, c, M.half_r, al, be, dx, dy, dz);
            const double ds = Aj.x - si;
            const double wax = al * dx, way = al * dy, waz = al * dz;
            // fused multiply-adds throughout: this kernel's bits need only
            // match themselves (batched and single launches)
            gx = fma(wax, ds, gx);
            gy0 = fma(way, ds, gy0);
            gz0 = fma(waz, ds, gz0);
            dv = fma(waz, fz + Bj.y, fma(way, fy + Bj.x, fma(wax, fx + Aj.y, dv)));
            const double tz = fma(pix, cj.x, fma(piy, cj.y, piz * cj.z)) -
                              fma(Cj.x, ci.x, fma(Cj.y, ci.y, Dj.x * ci.z));
            zt = fma(be, tz, zt);
            const double lxj[4] = {e0.x, e0.y, e1.x, e1.y};
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) d[bb] = fma(c, lxj[bb] - lxo[bb], d[bb]);
        }
        gx = grp_sum<L>(gx);
        gy0 = grp_sum<L>(gy0);
        gz0 = grp_sum<L>(gz0);
        dv = grp_sum<L>(dv);
        zt = grp_sum<L>(zt);
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) d[bb] = grp_sum<L>(d[bb]);
        const double2 U0 = oU0[li], U1 = oU1[li], EE = oE[li], XX = oX[li];
        const double ux = U0.x, uy = U0.y, uz = U1.x;
        const double xx = XX.x, xy = XX.y, xz = U1.y;
        const double eta = EE.x, xh = EE.y;
        const double nx = ci.x, ny = ci.y, nz = ci.z;
        const double gr = nx * gx + ny * gy0 + nz * gz0;
        const double Gx = gx - gr * nx, Gy = gy0 - gr * ny, Gz = gz0 - gr * nz;
        const double pux = ny * uz - nz * uy, puy = nz * ux - nx * uz, puz = nx * uy - ny * ux;
        const double pxx = ny * xz - nz * xy, pxy = nz * xx - nx * xz, pxz = nx * xy - ny * xx;
        double o[4];
        o[0] = sc * (-zt * pux - eta * pxx - Gx - nu * d[0]);
        o[1] = sc * (-zt * puy - eta * pxy - Gy - nu * d[1]);
        o[2] = sc * (-zt * puz - eta * pxz - Gz - nu * d[2]);
        o[3] = sc * (-dv - nu * d[3]);
        const double xs[4] = {xx, xy, xz, xh};
#pragma unroll
        for (int kc = 0; kc < kCompIter<L>; ++kc) {
            const int bb = comp_of<L>(q, kc);
            const int oi = 4 * i + bb;
            double ob = o[bb];
            if constexpr (EPI != kEpiIom2) {   // IOM2 columns carry no sum terms
#pragma unroll
                for (int k = 0; k < kPmax; ++k)
                    if (k < a.naxpy) ob += cax[k] * axv[k][oi];
            }
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

// Conserved quantities monitored in Sec. 6: per block, in its cells'
// order, the partial sums of A h (mass), A (h |u|^2 / 2 + g h^2 / 2 +
// g h h_s) (total energy) and A (zeta + f)^2 / (2 h) (potential enstrophy);
// zeta + f is the absolute vorticity k_linearize forms.
template <int L>
__global__ void __launch_bounds__(256) k_diag(DevMesh M, const double *__restrict__ u,
                                              double *__restrict__ parts) {
    __shared__ double lds[16 * 3];
    const int n = M.n;
    const int q = threadIdx.x & (L - 1);
    double acc[3] = {0.0, 0.0, 0.0};
    for (CellRange r = block_cells<L>(n); r.i < r.end; r.i += r.step) {
        const int i = r.i;
        const Cell ci = load_cell(M.cen, i);
        double ui[4];
        load4(u, i, ui);
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < kSlotIter<L>; ++k) {
            const int s = slot_of<L>(q, k);
            if (s < 0) continue;
            const int e = 6 * i + s;
            const int j = M.nbr[e];
            const Cell cj = load_cell(M.cen, j);
            const EdgeW w = edge_weights(ci, cj, M.alpha[e]);
            double uj[4];
            load4(u, j, uj);
            z = acc_add(z, w.bx * (ui[0] + uj[0]) + w.by * (ui[1] + uj[1]) + w.bz * (ui[2] + uj[2]));
        }
        z = grp_sum<L>(z);
        if (q == 0) {
            const double A = 1.0 / ci.ra, h = ui[3];
            const double sp2 = ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2];
            const double av = z + M.two_omega * ci.z;
            acc[0] += A * h;
            const double hs = M.hs ? M.hs[i] : 0.0;
            acc[1] += A * (0.5 * h * sp2 + 0.5 * M.g * h * h + M.g * h * hs);
            acc[2] += A * av * av / (2.0 * h);
        }
    }
    block_sum_all<3>(acc, lds);
    put_partials<3>(acc, parts);
}

// Totals of k_diag's partials, in block order, into out[0..2].
__global__ void __launch_bounds__(256) k_diag_sum(const double *__restrict__ parts, int np,
                                                  double *__restrict__ out) {
    __shared__ double lds[16 * 3];
    double t[3];
    sum_partials<3>(t, parts, np, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[k] = t[k];
}

// Blocks that cover every chunk once: the chunk count rounded up to whole
// XCDs (no die's share in xcd_chunks exceeds ceil(nchunks / 8)).
int lds_grid_cap(const DevMesh &M) { return (M.halo.nchunks + kXcd - 1) / kXcd * kXcd; }

// Whether a product launch takes k_jv_lds: a grid with chunk tables, two
// lanes per cell, a linearisation record to stage (every forward product of
// the library passes one), and no sum terms on an IOM2 column (none of the
// callers adds them there).
bool jv_uses_lds(const DevMesh &M, const JvArgs &a, int epi, int L) {
    return M.halo.nchunks > 0 && L == kJvLdsL && a.rec && red_parts(M.n) % kXcd == 0 &&
           !(epi == kEpiIom2 && a.naxpy > 0);
}

// Returns the number of partials the launch writes per member (0 without an
// epilogue).
template <int L, bool FL>
int jv_launch_t(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    if (jv_uses_lds(M, a, epi, L)) {
        // no more blocks than chunks (rounded to whole XCDs): a batched launch
        // would otherwise dispatch every member's empty blocks; norm partials
        // keep red_parts(n) blocks, the count their consumers sum
        const int cap = lds_grid_cap(M);
        const int np = epi == kEpiNorm ? red_parts(M.n) : (cap < red_parts(M.n) ? cap : red_parts(M.n));
        const dim3 grid(np, b.nm), block(kJvLdsBlock);
        const bool t4 = M.halo.short_terms == 4;
        if (epi == kEpiIom2) {
            if (t4) hipLaunchKernelGGL((k_jv_lds<kEpiIom2, 4>), grid, block, 0, s, M, a, b);
            else hipLaunchKernelGGL((k_jv_lds<kEpiIom2, kShortTerms>), grid, block, 0, s, M, a, b);
        } else if (epi == kEpiNorm) {
            if (t4) hipLaunchKernelGGL((k_jv_lds<kEpiNorm, 4>), grid, block, 0, s, M, a, b);
            else hipLaunchKernelGGL((k_jv_lds<kEpiNorm, kShortTerms>), grid, block, 0, s, M, a, b);
        } else {
            if (t4) hipLaunchKernelGGL((k_jv_lds<kEpiNone, 4>), grid, block, 0, s, M, a, b);
            else hipLaunchKernelGGL((k_jv_lds<kEpiNone, kShortTerms>), grid, block, 0, s, M, a, b);
        }
        return epi == kEpiNone ? 0 : np;
    }
    if (epi == kEpiNone) {
        hipLaunchKernelGGL((k_jv<kEpiNone, L, FL, false>), dim3(cells_grid(M.n, 256, L), b.nm), dim3(256),
                           0, s, M, a, b);
        return 0;
    }
    const int grid = red_parts(M.n);
    int block = red_block(M.n, b.nm, L);
    if (red_cells(M.n) <= kCellRedMax) {   // per-cell reduction: any block size gives the same bits
        const int want = (long)b.nm * M.n > 200000L ? M.jv_block_batch : M.jv_block;
        if (want > 0) block = want;
    }
    if (epi == kEpiIom2) {
        if (red_cells(M.n) <= kCellRedMax)
            hipLaunchKernelGGL((k_jv<kEpiIom2, L, FL, true>), dim3(grid, b.nm), dim3(block), 0, s, M, a, b);
        else
            hipLaunchKernelGGL((k_jv<kEpiIom2, L, FL, false>), dim3(grid, b.nm), dim3(block), 0, s, M, a, b);
    } else {
        const int nb = block < kJvMaxBlock<kEpiNorm> ? block : kJvMaxBlock<kEpiNorm>;
        if (red_cells(M.n) <= kCellRedMax)
            hipLaunchKernelGGL((k_jv<kEpiNorm, L, FL, true>), dim3(grid, b.nm), dim3(nb), 0, s, M, a, b);
        else
            hipLaunchKernelGGL((k_jv<kEpiNorm, L, FL, false>), dim3(grid, b.nm), dim3(nb), 0, s, M, a, b);
    }
    return grid;
}

template <int L>
int jv_launch(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    if constexpr (L == 8) {
        if (jv_fuses_lap(M, b.nm)) return jv_launch_t<8, true>(M, a, epi, b, s);
    }
    return jv_launch_t<L, false>(M, a, epi, b, s);
}

}  // namespace

void launch_lap4(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s) {
    const int L = launch_lanes(M, b.nm);
    if (M.halo.nchunks > 0 && L == kLapLdsL) {
        // four blocks per CU by default, XCD-major chunk sweep, and no more
        // blocks than chunks (both multiples of the XCD count)
        const int want = M.lap_grid > 0 ? M.lap_grid : 4 * 256;
        const int cap = lds_grid_cap(M);
        const int grid = want < cap ? want : cap;
        hipLaunchKernelGGL(k_lap4_lds, dim3(grid, b.nm), dim3(kLapLdsBlock), 0, s, M, psi, out, b);
        return;
    }
    const int lb = M.lap_block > 0 ? M.lap_block : 256;
#define XRB_CALL(L) \
    hipLaunchKernelGGL(k_lap4<L>, dim3(cells_grid(M.n, lb, L), b.nm), dim3(lb), 0, s, M, psi, out, b)
    XRB_LANES_DISPATCH_N(launch_lanes(M, b.nm), XRB_CALL)
#undef XRB_CALL
}

bool iom2_chunked(const DevMesh &M, int nm) {
    return M.halo.nchunks > 0 && launch_lanes(M, nm) == kUpdLapL && !jv_fuses_lap(M, nm);
}

bool upd_lap_fused(const DevMesh &M, int nm) { return nm == 1 && iom2_chunked(M, nm); }

namespace {
bool norm_per_chunk(const DevMesh &M) { return M.halo.nchunks <= kNrmRegion; }
// the grid both chunked forms take when their partials are per block: every
// chunk swept by kRedBlocks blocks (a multiple of the XCD count)
constexpr int kChunkedGrid = kRedBlocks;
}  // namespace

int chunked_norm_parts(const DevMesh &M) { return norm_per_chunk(M) ? M.halo.nchunks : kChunkedGrid; }

void launch_upd_lap(const DevMesh &M, int j, const double *w, const double *rj, const double *rjm1,
                    double *rn, double *lapn, PhiCtl *ctl, const double *nrm_in, int np_nrm,
                    const double *dot_in, int np_dot, double *nrm_out, const Batch &b, hipStream_t s) {
    // per-chunk partials: one chunk per block (whole XCDs); else the shared grid
    const int pc = norm_per_chunk(M);
    const int grid = pc ? lds_grid_cap(M) : kChunkedGrid;
    hipLaunchKernelGGL(k_upd_lap_lds, dim3(grid, b.nm), dim3(kUpdLapBlock), 0, s, M, j, w, rj, rjm1, rn,
                       lapn, ctl, nrm_in, np_nrm, dot_in, np_dot, nrm_out, pc, b);
}

void launch_iom2_update_lds(const DevMesh &M, int j, double *w, const double *rj, const double *rjm1,
                            PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                            int np_dot, double *nrm_out, const Batch &b, hipStream_t s) {
    // per-chunk partials: the streaming update's block count (about 4096
    // values per block, so that each block's prologue serves a few chunks) in
    // whole XCDs, at most one block per chunk; else the shared grid
    const int pc = norm_per_chunk(M);
    int grid = kChunkedGrid;
    if (pc) {
        const int cap = lds_grid_cap(M);
        grid = upd_parts(M.n) / kXcd * kXcd;
        grid = grid < kXcd ? kXcd : grid;
        grid = grid < cap ? grid : cap;
    }
    hipLaunchKernelGGL(k_iom2_update_lds, dim3(grid, b.nm), dim3(kUpdLapBlock), 0, s, M, j, w, rj, rjm1,
                       ctl, nrm_in, np_nrm, dot_in, np_dot, nrm_out, pc, b);
}

void launch_linearize(const DevMesh &M, const double *u, double *eta, double *rec, const Batch &b,
                      hipStream_t s) {
#define XRB_CALL(L) \
    hipLaunchKernelGGL(k_linearize<L>, dim3(cells_grid(M.n, 256, L), b.nm), dim3(256), 0, s, M, u, eta, rec, b)
    XRB_LANES_DISPATCH_N(launch_lanes(M, b.nm), XRB_CALL)
#undef XRB_CALL
}

void launch_rhs(const DevMesh &M, const double *u, const double *lu, double *f, const Batch &b,
                hipStream_t s) {
#define XRB_CALL(L) \
    hipLaunchKernelGGL(k_rhs<L>, dim3(cells_grid(M.n, 256, L), b.nm), dim3(256), 0, s, M, u, lu, f, b)
    XRB_LANES_DISPATCH_N(launch_lanes(M, b.nm), XRB_CALL)
#undef XRB_CALL
}

void launch_diag(const DevMesh &M, const double *u, double *parts, double *out, hipStream_t s) {
    const int grid = red_parts(M.n);
#define XRB_CALL(L) hipLaunchKernelGGL(k_diag<L>, dim3(grid), dim3(256), 0, s, M, u, parts)
    XRB_LANES_DISPATCH(XRB_CALL)
#undef XRB_CALL
    hipLaunchKernelGGL(k_diag_sum, dim3(1), dim3(256), 0, s, parts, grid, out);
}

int launch_jv(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s) {
    int np = 0;
#define XRB_CALL(L) np = jv_launch<L>(M, a, epi, b, s)
    XRB_LANES_DISPATCH_N(launch_lanes(M, b.nm), XRB_CALL)
#undef XRB_CALL
    return np;
}

}  // namespace xrb
