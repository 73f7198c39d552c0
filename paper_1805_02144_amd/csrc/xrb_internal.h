// Internal declarations of libexprb (HIP, gfx950).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/exprb.h"

namespace xrb {

constexpr int kBlock = 256;                               // threads per block, 4 waves
constexpr int kMmax = XRB_MMAX_LIMIT;                     // largest Krylov size
constexpr int kPmax = XRB_PMAX;
constexpr int kKmax = kMmax + kPmax + 1;                  // augmented matrix order

// Geometry of the finite-volume operators, cell-major ([cell][slot], 6
// slots): the lanes that share a cell in the edge-parallel kernels read one
// contiguous record per array.  For the edge from cell i to neighbour j
// (unit centres x_i, x_j), x_j - x_i is exactly tangent at the edge midpoint
// direction, so the flux and circulation weights are
//   a = l n_e / (2 A_i)  = alpha (x_j - x_i),  alpha = l / (2 A_i |x_j - x_i|)
//   b = l t_e / (2 A_i)  = beta  (x_i x x_j),  beta  = 2 alpha / |x_i + x_j|
// and the Laplacian weight is c = l / (d A_i).  alpha and c are stored per
// edge slot; the kernels form beta from alpha and the two centres they load
// (the LDS-staged kernels form alpha and beta from c and the chord by a
// short series: see edge_weights_short and edge_ab_short).
//
// Grids above 16384 cells (where the stencils default to two lanes per cell)
// also carry the chunk tables of the LDS-staged product and Laplacian: the
// cells are cut into chunks of kChunk consecutive cells; chunk k's one-ring
// halo (the neighbours outside the chunk, ascending) is hids[hoff[k] ..
// hoff[k+1]), and lnbr[6 i + s] is the position of slot s's neighbour in the
// chunk's staging order (the chunk's cells, then its halo).
constexpr int kChunk = 256;       // cells per chunk of the LDS-staged product
constexpr int kHaloMax = 128;     // largest halo the product's LDS holds
struct Halo {
    const int32_t *hoff = nullptr;   // [nchunks + 1]
    const int32_t *hids = nullptr;   // halo cell ids, chunk after chunk
    const uint16_t *lnbr = nullptr;  // [n][6]
    int nchunks = 0;                 // 0: no tables (small grid, or a halo above kHaloMax)
    int short_terms = 5;             // terms of the LDS product's weight series (4 or 5)
};
struct DevMesh {
    int n = 0;
    const int32_t *nbr = nullptr;                  // [n][6]
    const double *alpha = nullptr;                 // [n][6]
    const double *cl = nullptr;                    // [n][6]
    const double *cen = nullptr;                   // [n][4]: unit centre x, y, z, 1 / cell area
    double nu = 0.0, g = 0.0;
    double two_omega = 0.0;                        // Coriolis f_i = two_omega * z_i
    double half_r = 0.0;                           // sphere radius / 2 (the short weight series)
    int lanes = 8;                                 // lanes per cell in the stencils (1, 2, 4, 8)
    int lanes_batch = 8;                           // lanes of forward launches over many cells
    // launch shapes the autotuner may set (0 = the built-in rule); none of
    // them changes any result bit
    int jv_block = 0, jv_block_batch = 0;          // threads of a product launch that reduces
                                                   // per-cell terms (grids up to 65536 cells)
    int lap_block = 0;                             // threads of a gather Laplacian launch
    int lap_grid = 0;                              // blocks of an LDS-staged Laplacian launch
    const double *hs = nullptr;                    // [n] surface topography h_s, null = flat
    const int32_t *perm = nullptr;                 // [n] the caller's number of internal cell p
    Halo halo;
};

// lanes per cell of the stencil kernels on an n-cell grid
int stencil_lanes(int n);
// lanes of a forward stencil launch over nm members (M.lanes or M.lanes_batch)
int launch_lanes(const DevMesh &M, int nm);
// whether lanes a (single states) and b (batches) give the same bits
bool lanes_pair_bitwise(const DevMesh &M, int a, int b);

// Decision of one substep attempt, read back by the host.
struct Decision {
    double tau_u;       // substep actually attempted
    double omega;       // t_out eps / (tau_u Tol)
    double t;           // time after the attempt
    int32_t accept;     // 1 = accepted
    int32_t lands;      // 1 = tau_u landed exactly on the output time
    int32_t m_next;     // Krylov size of the next attempt
    int32_t m_eff;      // basis size used (breakdown may shorten it)
    int32_t status;     // 0 or an xrb_status
    int32_t reached;    // t == t_out after the attempt
    int32_t seq;        // host copy only: the attempt's sequence number, stored last
};

// Device-resident state of one phi_combo evaluation.
struct PhiCtl {
    double H[(kMmax + 1) * kMmax];   // IOM2 Hessenberg (banded), row-major
    double sigma[kMmax + 2];         // v_k = sigma[k] * R_k (raw basis scale)
    double beta;                     // ||w_p||
    int32_t brk;                     // breakdown: basis size, 0 = none
    int32_t beta_zero;               // beta == 0
    // controller state
    double t, t_out, tau, q, kappa, prev_tau, prev_omega, tol_abs;
    int32_t m, prev_m, have_prev, pad0;
    double rec_coef[kPmax + 1];      // t^l / l! at the current point
    double ycoef[kPmax + kMmax + 2]; // combine coefficients of an accepted attempt
    Decision dec;
    double pad[6];                   // keeps sizeof a multiple of 64 bytes
};

// Replay entry or sentinel passed to the controller kernel.
struct ReplayIn {
    double tau;
    int32_t m;
    int32_t flags;
    int32_t active;
};

// ---------------- batching ----------------
// Every kernel runs over nm members (member k = blockIdx.y).  Vector
// arguments of member k are the member-0 pointer plus k * ws doubles, the
// phi state is ctl + k, reduction partials are offset by k * kPartStride.
// A launch may carry a per-member predicate read from a plan table that the
// host uploads once per round; members for which it is false return at once.
enum PlanField {
    PF_IOM2_LO = 0,   // IOM2 column j runs iff plan[lo] <= j < plan[hi]
    PF_IOM2_HI = 1,
    PF_REC_PROD = 2,  // bit (j-1): w_j of the recurrence needs the product A w_{j-1}
    PF_REC_SUM = 3,   // bit (j-1): w_j is a pure sum of input terms
    PF_CTL = 4,       // member attempts a substep this round
    PF_COMB = 5,      // member accepted: combine
    PF_COPY = 6,      // member reached an output time: copy y out (value = slot + 1)
    PF_INIT = 7,      // member starts this phi evaluation
    kPlanW = 8
};
constexpr int kRedBlocks = 512;                    // cap on blocks (partials) of a reduction
// IOM2 column norms: two partial buffers per member (columns alternate), each
// room for one partial per block of an update or per chunk (chunked updates
// on grids of at most kNrmRegion chunks)
constexpr int kNrmRegion = kRedBlocks;
constexpr int kPartStride = 2 * kNrmRegion;        // per-member doubles: dot or norm partials
constexpr int kVPartStride = (kPmax + 1) * kRedBlocks;   // per-member doubles: input norms

// blocks of a reducing kernel over `items` work items, `block` per block
inline int red_grid(int items, int block) {
    int g = (items + block - 1) / block;
    if (g < 1) g = 1;
    return g > kRedBlocks ? kRedBlocks : g;
}

// Every reducing kernel launches red_parts(n) blocks on an n-cell grid (so
// every producer of a partial family writes the same number of partials).
inline int red_parts(int n) { return red_grid(8 * n, 256); }

// Blocks of the IOM2 update (a streaming kernel over 4n values whose
// prologue sums the previous kernels' partials): about 4096 values per
// block, between 64 and kRedBlocks blocks.  Its norm partials form a family
// of this size, which the kernels that finish a column are told explicitly.
inline int upd_parts(int n) {
    const long g = (4L * n + 4095) / 4096;
    return (int)(g < 64 ? 64 : (g > kRedBlocks ? kRedBlocks : g));
}

template <class T>
__host__ __device__ inline T *member_ptr(T *p, int64_t stride, int k) {
    return p ? p + stride * k : p;
}
template <class T>
__device__ inline T *ctl_member(T *c, int k) {
    return c + k;
}
// a coefficient that lives inside member 0's PhiCtl, moved to member k's
__device__ inline const double *ctl_field(const double *p, int k) {
    return (const double *)((const char *)p + (size_t)k * sizeof(PhiCtl));
}

struct Pred {
    const int32_t *plan = nullptr;   // [nm][kPlanW]; nullptr = all members active
    int field = 0;
    int j = 0;
};

__device__ inline bool member_active(const Pred &p, int k) {
    if (!p.plan) return true;
    const int32_t *q = p.plan + kPlanW * k;
    switch (p.field) {
        case PF_IOM2_LO:
            return q[PF_IOM2_LO] <= p.j && p.j < q[PF_IOM2_HI];
        case PF_REC_PROD:
        case PF_REC_SUM:
            return ((q[p.field] >> (p.j - 1)) & 1) != 0;
        default:
            return q[p.field] != 0;
    }
}

struct Batch {
    int nm = 1;
    int64_t ws = 0;        // member stride of vector arguments (doubles)
    Pred pred;
    const double *dtk = nullptr;   // per-member step sizes (device), used where noted
};

// ---------------- kernel launchers (stream-ordered) ----------------
// Reductions: a reducing kernel writes one partial per block and its
// launcher returns the block count; the next kernel that needs the total
// sums those partials (see reduce.h).

// out = L psi (4 components), raw input
void launch_lap4(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s);
// eta = V.u + f; rec (nullable, 8 doubles per cell) receives the record
// (u, centre, eta) of every cell
void launch_linearize(const DevMesh &M, const double *u, double *eta, double *rec, const Batch &b,
                      hipStream_t s);
// f = F(u), needs lu = L u (4 components)
void launch_rhs(const DevMesh &M, const double *u, const double *lu, double *f, const Batch &b,
                hipStream_t s);

// Generic Jacobian product
//   out = dt_k * J(u) x  +  sum_k coef[k] * axv[k]
// (dt_k = b.dtk[member] when b.dtk is set, else a.dt)
// kEpiNone : plain.
// kEpiNorm : partials of ||out||^2 into nrm_out.
// kEpiIom2 : column j of IOM2 on the raw basis vector x = R_j: partials of
//            <out, R_j> and <out, R_{j-1}> into dot_out (the scales are
//            applied by the IOM2 update that follows).
enum JvEpi { kEpiNone = 0, kEpiIom2 = 1, kEpiNorm = 2 };
struct JvArgs {
    const double *u = nullptr;      // linearisation state
    const double *eta = nullptr;    // V.u + f
    // per-cell record (u_x, u_y, u_z, h, x, y, z, eta) of the linearisation
    // state, written by launch_linearize; nullable (then the products of
    // large grids read u, eta and the centres from their own arrays)
    const double *rec = nullptr;
    const double *x = nullptr;      // direction (raw)
    const double *lx = nullptr;     // L x (raw)
    double dt = 1.0;
    double *out = nullptr;
    int naxpy = 0;
    const double *axv[kPmax] = {};
    const double *axc[kPmax] = {};  // device pointers to coefficients, in PhiCtl of member 0
    // IOM2
    int j = 0;
    const double *rjm1 = nullptr;
    PhiCtl *ctl = nullptr;
    double *dot_out = nullptr;
    double *nrm_out = nullptr;
};
// When jv_fuses_lap(M, b.nm) holds the product forms L x itself and ignores
// a.lx, so callers skip the launch_lap4 pass that would feed it; the two
// forms give the same bits.
bool jv_fuses_lap(const DevMesh &M, int nm);
int launch_jv(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s);
// IOM2 columns of a launch over nm members on a grid with chunk tables (two
// lanes, the product not forming L x itself) take the chunked update, in one
// of two forms with the same bits.  Single states take launch_upd_lap, the
// update fused with the next column's Laplacian: the product writes w to a
// buffer of its own, and the kernel forms R_{j+1} into rn and L R_{j+1} into
// lapn.  Batches take launch_iom2_update_lds (R_{j+1} over w in place; the
// next column's Laplacian is its own pass), which overlaps better across
// members.  The column norm's partials (chunked_norm_parts(M) of them, the
// count every consumer of an IOM2 column's norm is told) are one per chunk
// on grids of at most kNrmRegion chunks, so that the two forms may take
// different grids, and otherwise one per block of kRedBlocks blocks that
// both forms take, sweeping the same chunks in the same order.
bool iom2_chunked(const DevMesh &M, int nm);
bool upd_lap_fused(const DevMesh &M, int nm);
int chunked_norm_parts(const DevMesh &M);
void launch_upd_lap(const DevMesh &M, int j, const double *w, const double *rj, const double *rjm1,
                    double *rn, double *lapn, PhiCtl *ctl, const double *nrm_in, int np_nrm,
                    const double *dot_in, int np_dot, double *nrm_out, const Batch &b, hipStream_t s);
void launch_iom2_update_lds(const DevMesh &M, int j, double *w, const double *rj, const double *rjm1,
                            PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                            int np_dot, double *nrm_out, const Batch &b, hipStream_t s);

// out = sum_k coef[k] * vec[k] (coefficients inside PhiCtl, offset per member);
// nrm_out (nullable) receives partials of ||out||^2
int launch_lincomb_dev(int n, double *out, int k, const double *const *vec,
                       const double *const *coef, PhiCtl *ctl0, double *nrm_out,
                       const Batch &b, hipStream_t s);
// Mass, total energy and potential enstrophy of the cell-major state u into
// out[0..2] (device); parts holds 3 red_parts(n) partials.
void launch_diag(const DevMesh &M, const double *u, double *parts, double *out, hipStream_t s);
// Caller layout [u_x | u_y | u_z | h] (component-major, the caller's cell
// numbers) to the kernels' cell-major [cell][4] in their own cell order
// (to_cell: internal cell p takes the caller's cell perm[p]) or back, for nm
// members at strides ss / ds (doubles); src and dst must not overlap.
void launch_relayout(int n, const int32_t *perm, int nm, const double *src, int64_t ss, double *dst,
                     int64_t ds, bool to_cell, hipStream_t s);
// out = sum_i c[i] * vec[i] (c[i] times dt_k when bit i of dtmask is set), length n4
void launch_lincomb(int n4, double *out, int k, const double *const *vec, const double *c,
                    unsigned dtmask, const Batch &b, hipStream_t s);
// IOM2 update of column j.  Prologue: finalise the column scale sigma_j from
// the norm partials of R_j (beta for j = 0, else h_{j,j-1} with the
// breakdown test), then H[j][j] = sigma_j^2 <w, R_j>, H[j-1][j] =
// sigma_j sigma_{j-1} <w, R_{j-1}> from the dot partials.  Body:
// R_{j+1} = sigma_j w - H[j][j] sigma_j R_j - H[j-1][j] sigma_{j-1} R_{j-1}
// (w = dt J R_j is stored in the R_{j+1} slot), norm partials to nrm_out.
// nrm_in and nrm_out are different buffers (ping-pong).
int launch_iom2_update(int n, int j, double *rjp1, const double *rj, const double *rjm1,
                       PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                       int np_dot, double *nrm_out, const Batch &b, hipStream_t s);
// y = sum_{j<p, !wzero} ycoef[j] w_j + sum_{k<meff} ycoef[p+k] R_k + ycoef[p+meff] R_meff
// (meff read from the member's decision)
void launch_combine(int n4, double *y, int p, const double *const *w, const int *wzero,
                    const double *V, PhiCtl *ctl, const Batch &b, hipStream_t s);
// partials of ||vec_k||^2, k < nv (<= kPmax+1), into parts[b*nv + k]
int launch_norms(int n, int nv, const double *const *vec, double *parts, const Batch &b,
                 hipStream_t s);
// out_slot[plan[PF_COPY]-1] <- y for members whose plan[PF_COPY] > 0
void launch_copy_out(int n4, const double *y, double *const *slots, const Batch &b,
                     hipStream_t s);

struct CtlArgs {
    int m;                // Krylov size requested for this attempt
    int p;
    int mode;             // FREE / RECORD / REPLAY
    int m_max;
    int wp_zero;          // w_p is the zero vector (symbolic)
    int built;            // IOM2 columns built at this point
    int nrm_buf;          // which norm-partials buffer holds the last column's norm
    int n_nrm_in;         // number of those partials
    double t_out;         // output time of this substep
    double n4;            // vector length (cost model)
    double delta, gamma;
    ReplayIn rep;
};
// Small augmented-Hessenberg exponential + error estimate + (tau, m) controller
// for the current attempt; writes ctl->dec and, on accept, the combine
// coefficients and the next point's recurrence coefficients.  The same record
// goes to hdec[k] (pinned host memory mapped on the device) followed by a
// system-scope release store of `seq` into hdec[k].seq, so the host may read
// the record as soon as it sees that number, without a stream synchronisation.
// Per-member arguments come from `dargs` (device, [nm]) when set, else from `a`.
void launch_controller(PhiCtl *ctl, const CtlArgs &a, const CtlArgs *dargs, double *nrm_parts,
                       Decision *hdec, int seq, const Batch &b, hipStream_t s);
// Initialise a call: t = 0, tau = rho_1, m, q, kappa, tol_abs from the norm
// partials of the nv input vectors; vnorm2[k*(kPmax+1) + l] = ||v_l||^2.
// m0 per member from m0k (device, [nm]) when set, else m0.
void launch_phi_init(PhiCtl *ctl, int m0, const int32_t *m0k, double tau0, double tol_rel,
                     const double *parts, int np, int nv, double *vnorm2, const Batch &b,
                     hipStream_t s);

// ---------------- adjoint (vector-Jacobian product) path ----------------
// acc (= or +=) scale * sum_{r < R} coef_r K(a0 + r sa, b0 + r sb)
struct KPairArgs {
    const double *a0 = nullptr;
    int64_t sa = 0;
    const double *b0 = nullptr;
    int64_t sb = 0;
    int R = 0;
    const double *coef = nullptr;   // device [R], nullptr = all 1
    double scale = 1.0;
    double *out = nullptr;
    int accumulate = 0;
};
constexpr int kMultiOut = kPmax + 1;       // mu_k and vbar_1..vbar_p
constexpr int kCoefLd = kMmax + 2;         // coefficients per output row
struct MultiArgs {
    int nout = 0;
    double *out[kMultiOut] = {};
    unsigned accmask = 0;
    int nv = 0;
    const double *vbase = nullptr;
    int64_t vstride = 0;
    const double *C = nullptr;              // device [nout][kCoefLd]
};
constexpr int kZRows = kMmax + 1;          // adjoint basis vectors
constexpr int kZLd = kMmax + 1 + kPmax;    // forward substep solution basis
struct ZArgs {
    int na = 0, nb = 0;
    const double *w[kZLd] = {};
    const double *z = nullptr;              // device [kZRows][kZLd]
    double *Z = nullptr;
    int64_t zstride = 0;
};
constexpr int kBigMax = 96;                 // >= kZRows + kZLd: the Van Loan block size
constexpr int kBigLd = kBigMax + 1;
struct AdjGArgs {
    int m = 0, built = 0, p = 0;
    double tau = 0.0, t = 0.0, t_out = 0.0, tol_abs = 0.0;
    const double *nrm_in = nullptr;
    int np = 0;
};
struct AdjOut {
    double omega;
    int32_t me, brk, beta_zero, status;
};
struct AdjVArgs {
    int me = 0, my = 0, p = 0;
    double tau = 0.0;
    int wzero = 0;                          // bit j: w_j of the forward substep is zero
};
void launch_lapT(const DevMesh &M, const double *psi, double *out, const Batch &b, hipStream_t s);
int launch_jtv(const DevMesh &M, const JvArgs &a, int epi, const Batch &b, hipStream_t s);
void launch_kpairs(const DevMesh &M, const KPairArgs &k, const Batch &b, hipStream_t s);
void launch_lincomb_multi(int n4, const MultiArgs &a, const Batch &b, hipStream_t s);
void launch_zgemm(int n4, const ZArgs &a, hipStream_t s);
void launch_adj_gexp(PhiCtl *c, const AdjGArgs &a, double *mat, double *work, double *C,
                     AdjOut *out, hipStream_t s);
void launch_adj_vanloan(const PhiCtl *c, const PhiCtl *cy, const AdjVArgs &a, double *mat,
                        double *work, double *z, hipStream_t s);

// ---------------- host geometry ----------------
struct HostGeometry {
    int n = 0;
    std::vector<int32_t> nbr;                              // [n][6]
    std::vector<double> alpha, cl;                         // [n][6]
    std::vector<double> cen;                               // [n][4] x, y, z, 1 / area
    std::vector<double> area;                              // [n] cell areas (m^2)
    std::vector<int32_t> perm;                             // [n] caller's cell of internal cell p
    double nu = 0.0;
    // chunk tables of the LDS-staged product (see Halo); empty when unused
    std::vector<int32_t> hoff, hids;
    std::vector<uint16_t> lnbr;
    int short_terms = 5;   // terms of the product's weight series (see Halo)
};
// Validates the mesh, picks the kernels' cell order (geo.perm: recursive
// coordinate bisection into kChunk-cell patches) and derives every per-cell
// and per-edge array in that order.
int build_geometry(const xrb_mesh &mesh, const xrb_params &prm, HostGeometry &geo,
                   std::string &err);
// Chunk tables for grids whose products take the LDS-staged kernel; leaves
// them empty when a chunk's halo exceeds kHaloMax or two neighbours lie
// beyond the range of the short weight series, and sets short_terms to four
// when every half-chord is within the four-term range.
void build_halo(HostGeometry &geo);

}  // namespace xrb
