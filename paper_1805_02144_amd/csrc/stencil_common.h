// Device helpers shared by the forward and transposed stencil kernels:
// lane groups, DPP group sums, cell records, edge weights, XCD-aware cell
// ranges and the lanes-per-cell dispatch.
#pragma once
#include "xrb_internal.h"

namespace xrb {
namespace stc {


constexpr int kXcd = 8;   // accelerator dies, each with its own L2

// The chunks [first, end) of the LDS-staged kernels that the blocks on die x
// sweep (blocks b with b % kXcd == x, the hardware's round-robin): the chunk
// count split over the dies as evenly as possible, the larger shares on the
// last dies.  A die with one chunk more than its blocks' even share then
// gives the extra step to the block that also takes the grid's last chunk,
// which may hold a few cells only (2561 chunks over 512 blocks: 5 steps
// everywhere but one block's sixth, two-cell chunk).
struct ChunkSpan {
    int first, end;
};
__device__ inline ChunkSpan xcd_chunks(int nchunks, int xcd) {
    const int base = nchunks / kXcd, from = kXcd - nchunks % kXcd;
    const int first = xcd * base + (xcd > from ? xcd - from : 0);
    return {first, first + base + (xcd >= from ? 1 : 0)};
}

// one block per block/L cells, rounded up to a whole number of blocks per XCD
inline int cells_grid(int n, int block, int L) {
    const int cpb = block / L;
    int g = (n + cpb - 1) / cpb;
    if (g < 1) g = 1;
    return (g + kXcd - 1) / kXcd * kXcd;
}

// Block size of a reducing stencil launch: the partial count is fixed by
// red_parts(n), so larger grids get wider blocks (more waves per CU) rather
// than more partials; small ones keep 256 threads and a few iterations.
inline int red_block(int n) { return n > 65536 ? 1024 : 256; }

// Cells per block of a reducing stencil launch (red_parts(n) blocks): at
// most kCellRedMax for n <= 65536, where the kernels reduce per-cell terms
// in a fixed order that does not depend on the block size.
constexpr int kCellRedMax = 128;
inline int red_cells(int n) {
    const int g = red_parts(n);
    return (n + g - 1) / g;
}

// Block size of a reducing product launch over nm members with L lanes per
// cell: with per-cell reduction the block size is free, so a launch takes the
// fewest whole waves that cover its chunk in one pass, at most 512 threads for
// a launch over few cells in all on a grid above 16384 cells (latency) and 256
// otherwise (throughput).  A level-6 chunk of 81 cells on two lanes fills 162
// of 192 threads (fewer idle lanes than 256 in batches, and at least as fast
// as 512 for a single state).
inline int red_block(int n, int nm, int L) {
    const int per = red_cells(n);
    if (per > kCellRedMax) return red_block(n);
    const int cap = ((long)nm * n <= 200000L && n > 16384) ? 512 : 256;
    const int b = (per * L + 63) / 64 * 64;
    return b < cap ? b : cap;
}

// Lane exchange inside a row by a DPP control word (VALU, no LDS traffic).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the L lanes of a cell: for eight, half-row mirror (lane i with
// 7-i) first; then xor 1 and xor 2 inside each quad.  Every lane ends with
// the same operands added in the same pairs (only commuted), so the L
// results are bitwise identical.
//
// Lane placement.  Lane q of L serves the edge slots slot_of<L>(q, k) and
// writes the output components comp_of<L>(q, k), k < kSlotIter<L> /
// kCompIter<L> (a negative value: none).  For L = 1, 2, 4 these are
// q, q + L, ...  For L = 8 the six slots sit on lanes 0, 2, 7, 5, 1, 3 and
// the four components on lanes 0, 2, 7, 5, so that grp_sum<8> adds them in
// the pairs ((s0 + s2) + s4) + ((s1 + s3) + s5) and (c0 + c2) + (c1 + c3):
// exactly what two lanes' running sums and one xor-1 exchange give.  With
// the edge and component sums accumulated without contraction (acc_add),
// the two- and eight-lane kernels therefore produce the same bits, and a
// launch may take either.
template <int L>
constexpr int kSlotIter = (6 + L - 1) / L;
template <int L>
constexpr int kCompIter = (4 + L - 1) / L;
template <int L>
__device__ inline int slot_of(int q, int k) {
    if (L == 8) {
        const int v = (0x2F3F5140 >> (4 * q)) & 0xF;   // lane -> slot, F = none
        return v == 0xF ? -1 : v;
    }
    const int s = q + L * k;
    return s < 6 ? s : -1;
}
template <int L>
__device__ inline int comp_of(int q, int k) {
    if (L == 8) {
        const int v = (0x2F3FF1F0 >> (4 * q)) & 0xF;   // lane -> component, F = none
        return v == 0xF ? -1 : v;
    }
    const int b = q + L * k;
    return b < 4 ? b : -1;
}

// a + t rounded on its own (never fused with the product that formed t)
__device__ inline double acc_add(double a, double t) {
#pragma clang fp contract(off)
    return a + t;
}
template <int L>
__device__ inline double grp_sum(double v) {
    if (L >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
    if (L >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    if (L >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    return v;
}

// Cell record: unit centre and reciprocal area, two 16-byte loads.  The
// Coriolis parameter is rebuilt as (2 Omega) z, the same product the host
// geometry forms.
struct Cell {
    double x, y, z, ra;
};
__device__ inline Cell load_cell(const double *__restrict__ cen, int i) {
    const double2 *p = reinterpret_cast<const double2 *>(cen) + 2 * (size_t)i;
    const double2 a = p[0], b = p[1];
    return {a.x, a.y, b.x, b.y};
}

// State and Krylov vectors are stored cell-major, [cell][4] = (u_x, u_y, u_z,
// h): component b of cell i sits at 4 i + b, and a gathered neighbour's four
// components come in two 16-byte loads (vectors start 16-byte aligned).
__device__ inline void load4(const double *__restrict__ v, int i, double (&o)[4]) {
    const double2 *p = reinterpret_cast<const double2 *>(v) + 2 * (size_t)i;
    const double2 a = p[0], b = p[1];
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
}

// The flux and circulation weights of the edge i -> j rebuilt from its
// Laplacian weight c = l / (d A_i) and the two unit centres alone.  With the
// chord 2y = |x_j - x_i| and the great-circle distance d = 2 a asin(y) (a the
// sphere radius), alpha = l / (2 A_i |x_j - x_i|) = c (a / 2) asin(y) / y;
// and since |x_i + x_j|^2 = 4 - |x_j - x_i|^2 on the unit sphere,
// beta = 2 alpha / |x_i + x_j| = alpha (1 - y^2)^(-1/2).  Both factors are
// series in y^2 summed by Horner over kShortTerms terms:
//   asin(y) / y = sum_k a_k y^(2k),  a_0 = 1, a_(k+1) = a_k (2k+1)^2 / ((2k+2)(2k+3))
//   (1 - y^2)^(-1/2) = sum_k b_k y^(2k),  b_0 = 1, b_(k+1) = b_k (2k+1) / (2k+2)
// For y^2 <= kShortY2Max (neighbour angles up to 2.3 degrees; level 6 of the
// icosahedral grid has 1.2) the first omitted terms are below 3e-18 of the
// sums, so these weights agree with the stored alpha and the square-root
// form of beta to rounding.  The LDS-staged product uses them (no alpha
// stream, no square root); the host enables that product only on grids
// inside the series' range.  Four terms suffice for y^2 <= kShort4Y2Max
// (the first omitted term, b_4 y^8, is below 3e-19; levels 7 and 8 have
// y^2 up to 2.7e-5 and 7e-6): the host picks the term count per grid.
constexpr int kShortTerms = 5;
constexpr double kShortY2Max = 4e-4;
constexpr double kShort4Y2Max = 3e-5;
struct ShortSeries {
    double a[kShortTerms], b[kShortTerms];
};
constexpr ShortSeries short_series() {
    ShortSeries s{};
    s.a[0] = 1.0;
    s.b[0] = 1.0;
    for (int k = 0; k + 1 < kShortTerms; ++k) {
        s.a[k + 1] = s.a[k] * (double)((2 * k + 1) * (2 * k + 1)) / (double)((2 * k + 2) * (2 * k + 3));
        s.b[k + 1] = s.b[k] * (double)(2 * k + 1) / (double)(2 * k + 2);
    }
    return s;
}

// The edge's flux weight alpha (the a of EdgeW is alpha (x_j - x_i)), the
// circulation weight beta and x_j - x_i from c and the two centres by the
// first NT terms of the series above.
template <int NT>
__device__ inline void edge_ab_short(const Cell &ci, const Cell &cj, double c, double half_r,
                                     double &al, double &be, double &dx, double &dy, double &dz) {
    static_assert(NT >= 1 && NT <= kShortTerms, "series terms");
    constexpr ShortSeries S = short_series();
    dx = cj.x - ci.x;
    dy = cj.y - ci.y;
    dz = cj.z - ci.z;
    const double y2 = 0.25 * (dx * dx + dy * dy + dz * dz);
    double fa = S.a[NT - 1], fb = S.b[NT - 1];
#pragma unroll
    for (int k = NT - 2; k >= 0; --k) {
        fa = fa * y2 + S.a[k];
        fb = fb * y2 + S.b[k];
    }
    al = c * half_r * fa;
    be = al * fb;
}

// Flux and circulation weights of the edge i -> j rebuilt from its scalar
// alpha and the two unit centres: a = alpha (x_j - x_i) and
// b = beta (x_i x x_j) with beta = 2 alpha / |x_i + x_j| (the edge's
// circulation weight l t / (2 A_i)).  beta is evaluated without contraction,
// so every kernel and lane count forms the same bits.
struct EdgeW {
    double ax, ay, az, bx, by, bz;
};
__device__ inline double edge_beta(const Cell &ci, const Cell &cj, double al) {
#pragma clang fp contract(off)
    const double sx = ci.x + cj.x, sy = ci.y + cj.y, sz = ci.z + cj.z;
    const double s2 = (sx * sx + sy * sy) + sz * sz;
    return (2.0 * al) * rsqrt(s2);
}
__device__ inline EdgeW edge_weights(const Cell &ci, const Cell &cj, double al);
// the same from the edge's Laplacian weight c by the short series above
// (half_r = a / 2)
__device__ inline EdgeW edge_weights_short(const Cell &ci, const Cell &cj, double c, double half_r) {
    constexpr ShortSeries S = short_series();
    const double dx = cj.x - ci.x, dy = cj.y - ci.y, dz = cj.z - ci.z;
    const double y2 = 0.25 * (dx * dx + dy * dy + dz * dz);
    double fa = S.a[kShortTerms - 1], fb = S.b[kShortTerms - 1];
#pragma unroll
    for (int k = kShortTerms - 2; k >= 0; --k) {
        fa = fa * y2 + S.a[k];
        fb = fb * y2 + S.b[k];
    }
    const double al = c * half_r * fa;
    const double be = al * fb;
    EdgeW w;
    w.ax = al * dx;
    w.ay = al * dy;
    w.az = al * dz;
    w.bx = be * (ci.y * cj.z - ci.z * cj.y);
    w.by = be * (ci.z * cj.x - ci.x * cj.z);
    w.bz = be * (ci.x * cj.y - ci.y * cj.x);
    return w;
}
__device__ inline EdgeW edge_weights(const Cell &ci, const Cell &cj, double al) {
    const double be = edge_beta(ci, cj, al);
    EdgeW w;
    w.ax = al * (cj.x - ci.x);
    w.ay = al * (cj.y - ci.y);
    w.az = al * (cj.z - ci.z);
    w.bx = be * (ci.y * cj.z - ci.z * cj.y);
    w.by = be * (ci.z * cj.x - ci.x * cj.z);
    w.bz = be * (ci.x * cj.y - ci.y * cj.x);
    return w;
}

// Cells of this block: one contiguous chunk, walked block/L cells at a
// time.  Workgroups are dispatched round-robin over the XCDs (block b on
// XCD b mod 8); numbering the chunks XCD-major gives every XCD one
// contiguous eighth of the grid, swept in order, so the neighbour lines a
// block gathers were mostly brought into the same L2 by the blocks beside it.
struct CellRange {
    int i, end, step;
    int first;   // first cell of the block's chunk
};
template <int L>
__device__ inline CellRange block_cells(int n) {
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    const int chunk = (G % kXcd) ? b : (b % kXcd) * (G / kXcd) + b / kXcd;
    const int per = (n + G - 1) / G;
    const int i0 = chunk * per;
    const int i1 = i0 + per < n ? i0 + per : n;
    return {i0 + (int)threadIdx.x / L, i1, (int)blockDim.x / L, i0};
}

// Multi-pass variant for the reducing kernels on large grids: XCD x owns
// the cells [x per8, (x+1) per8), and its G/8 blocks sweep them together,
// pass by pass, in contiguous windows of (G/8) (block/L) cells -- so the
// lines the blocks of one XCD gather at any time lie in one window of the
// grid rather than under G/8 separate cursors.  Falls back to block_cells
// when G is not a multiple of 8.
template <int L>
__device__ inline CellRange block_cells_swept(int n) {
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    if (G % kXcd) return block_cells<L>(n);
    const int x = b % kXcd, k = b / kXcd, nb = G / kXcd;
    const int per8 = (n + kXcd - 1) / kXcd;
    const int x0 = x * per8;
    const int x1 = x0 + per8 < n ? x0 + per8 : n;
    const int cpb = (int)blockDim.x / L;
    return {x0 + k * cpb + (int)threadIdx.x / L, x1, nb * cpb, x0};
}

}  // namespace stc

#define XRB_LANES_DISPATCH_N(NL, CALL)      \
    switch (NL) {                           \
    case 1: CALL(1); break;                 \
    case 2: CALL(2); break;                 \
    case 4: CALL(4); break;                 \
    default: CALL(8); break;                \
    }

#define XRB_LANES_DISPATCH(CALL)            \
    switch (M.lanes) {                      \
    case 1: CALL(1); break;                 \
    case 2: CALL(2); break;                 \
    case 4: CALL(4); break;                 \
    default: CALL(8); break;                \
    }

}  // namespace xrb
