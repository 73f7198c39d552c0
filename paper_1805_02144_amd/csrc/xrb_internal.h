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
// slots): the eight lanes that share a cell in the edge-parallel kernels read
// one contiguous 48-byte record per array.
//   a_s = l_e n_{e,i} / (2 A_i)   divergence and gradient weights (3 comps)
//   b_s = l_e t_{e,i} / (2 A_i)   vorticity (circulation) weights (3 comps)
//   c_s = l_e / (d_e A_i)         Laplacian weights
struct DevMesh {
    int n = 0;
    const int32_t *nbr = nullptr;                  // [n][6]
    const double *ax = nullptr, *ay = nullptr, *az = nullptr;   // [n][6] each
    const double *bx = nullptr, *by = nullptr, *bz = nullptr;
    const double *cl = nullptr;                    // [n][6]
    const double *nx = nullptr, *ny = nullptr, *nz = nullptr;   // [n] cell normals
    const double *cor = nullptr;                   // [n] Coriolis 2 Omega sin(lat)
    double nu = 0.0, g = 0.0;
};

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
};

// Replay entry or sentinel passed to the controller kernel.
struct ReplayIn {
    double tau;
    int32_t m;
    int32_t flags;
    int32_t active;
};

// ---------------- kernel launchers (stream-ordered) ----------------
// Reductions: a reducing kernel writes one partial per block and its
// launcher returns the block count; the next kernel that needs the total
// sums those partials (see reduce.h).

// out = L psi (4 components), raw input
void launch_lap4(const DevMesh &M, const double *psi, double *out, hipStream_t s);
// eta = V.u + f
void launch_linearize(const DevMesh &M, const double *u, double *eta, hipStream_t s);
// f = F(u), needs lu = L u (4 components)
void launch_rhs(const DevMesh &M, const double *u, const double *lu, double *f, hipStream_t s);

// Generic Jacobian product
//   out = dt * J(u) x  +  sum_k coef[k] * axv[k]
// kEpiNone : plain.
// kEpiNorm : partials of ||out||^2 into nrm_out.
// kEpiIom2 : column j of IOM2 on the raw basis vector x = R_j: partials of
//            <out, R_j> and <out, R_{j-1}> into dot_out (the scales are
//            applied by the IOM2 update that follows).
enum JvEpi { kEpiNone = 0, kEpiIom2 = 1, kEpiNorm = 2 };
struct JvArgs {
    const double *u = nullptr;      // linearisation state
    const double *eta = nullptr;    // V.u + f
    const double *x = nullptr;      // direction (raw)
    const double *lx = nullptr;     // L x (raw)
    double dt = 1.0;
    double *out = nullptr;
    int naxpy = 0;
    const double *axv[kPmax] = {};
    const double *axc[kPmax] = {};  // device pointers to coefficients
    // IOM2
    int j = 0;
    const double *rjm1 = nullptr;
    PhiCtl *ctl = nullptr;
    double *dot_out = nullptr;
    double *nrm_out = nullptr;
};
int launch_jv(const DevMesh &M, const JvArgs &a, int epi, hipStream_t s);

// out = sum_k coef[k] * vec[k] (device coefficient pointers); nrm_out
// (nullable) receives partials of ||out||^2
int launch_lincomb_dev(int n, double *out, int k, const double *const *vec,
                       const double *const *coef, double *nrm_out, hipStream_t s);
// out = sum_k c[k] * vec[k], host coefficients (k <= 6), length n4
void launch_lincomb(int n4, double *out, int k, const double *const *vec, const double *c,
                    hipStream_t s);
// IOM2 update of column j.  Prologue: finalise the column scale sigma_j from
// the norm partials of R_j (beta for j = 0, else h_{j,j-1} with the
// breakdown test), then H[j][j] = sigma_j^2 <w, R_j>, H[j-1][j] =
// sigma_j sigma_{j-1} <w, R_{j-1}> from the dot partials.  Body:
// R_{j+1} = sigma_j w - H[j][j] sigma_j R_j - H[j-1][j] sigma_{j-1} R_{j-1}
// (w = dt J R_j is stored in the R_{j+1} slot), norm partials to nrm_out.
// nrm_in and nrm_out are different buffers (ping-pong).
int launch_iom2_update(int n, int j, double *rjp1, const double *rj, const double *rjm1,
                       PhiCtl *ctl, const double *nrm_in, int np_nrm, const double *dot_in,
                       int np_dot, double *nrm_out, hipStream_t s);
// y = sum_{j<p, !wzero} ycoef[j] w_j + sum_{k<meff} ycoef[p+k] R_k + ycoef[p+meff] R_meff
void launch_combine(int n4, double *y, int p, const double *const *w, const int *wzero,
                    const double *V, int meff, int corr, PhiCtl *ctl, hipStream_t s);
// partials of ||vec_k||^2, k < nv (<= kPmax+1), into parts[b*nv + k]
int launch_norms(int n, int nv, const double *const *vec, double *parts, hipStream_t s);

struct CtlArgs {
    int m;                // Krylov size requested for this attempt
    int p;
    int mode;             // FREE / RECORD / REPLAY
    int m_max;
    int wp_zero;          // w_p is the zero vector (symbolic)
    int built;            // IOM2 columns built at this point
    double n4;            // vector length (cost model)
    double delta, gamma;
    ReplayIn rep;
    const double *nrm_in; // partials of the last column's norm
    int n_nrm_in;
};
// Small augmented-Hessenberg exponential + error estimate + (tau, m) controller
// for the current attempt; writes ctl->dec and, on accept, the combine
// coefficients and the next point's recurrence coefficients.
void launch_controller(PhiCtl *ctl, const CtlArgs &a, hipStream_t s);
// Initialise a call: t = 0, tau = rho_1, m, q, kappa, tol_abs from the norm
// partials of the nv input vectors; vnorm2_out[k] = ||v_k||^2
void launch_phi_init(PhiCtl *ctl, int m0, double tau0, double tol_rel, const double *parts,
                     int np, int nv, double *vnorm2_out, hipStream_t s);
// Start a new output interval
void launch_set_tout(PhiCtl *ctl, double t_out, hipStream_t s);

// ---------------- host geometry ----------------
struct HostGeometry {
    int n = 0;
    std::vector<int32_t> nbr;                              // [n][6]
    std::vector<double> ax, ay, az, bx, by, bz, cl;        // [n][6]
    std::vector<double> nx, ny, nz, cor;                   // [n]
    double nu = 0.0;
};
int build_geometry(const xrb_mesh &mesh, const xrb_params &prm, HostGeometry &geo,
                   std::string &err);

}  // namespace xrb
