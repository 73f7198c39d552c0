/*
 * Plain CPU oracle for the exponential Rosenbrock / phipm_simul_iom2 hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never links, imports or calls it, and it shares no code with the HIP
 * library.
 *
 * Everything is FP64, serial, written as plain loops in the paper's order:
 *   - rotating shallow water right-hand side F(u)      (Sec. 2, eq. sweqsinv,
 *     dissipation eqs. swdis/niu)
 *   - Jacobian-vector product J(u)v = (J_v + J_r + J_m) v  (eqs. dynjs,
 *     dynja, dynjb, dynjc; row 2 of J_r read with the signs that the
 *     derivative of P_y = n_z u_x - n_x u_z gives)
 *   - transposed product J(u)^T w
 *   - Pade [13/13] scaling-and-squaring matrix exponential (used for the
 *     augmented Hessenberg exponential of Alg. 1, step 2)
 *   - phipm_simul_iom2 (Alg. 1, Sec. 4.3) with IOM2 and a (tau, m)
 *     controller of the shape the paper cites (constants stated in orc_phi.c)
 *   - exprb42, pexprb43, exprb53 (eqs. 3.11-3.13), epi3 (eq. epi3) with an
 *     EPI2 starting step (eq. 3.5), through the call mapping of Sec. 4.4.
 *   - the adjoint (not in the paper): K(a, b) = grad_u <a, J(u) b>, the
 *     continuous adjoint of one phi-combination on the substeps of its
 *     forward solve (orc_adjoint.c states the construction), and the
 *     vector-Jacobian product of one exprb42 step.
 *
 * Parity status: the controller of Alg. 1 (steps 4-5) is only cited by the
 * paper; its constants are a reading ("parity unpinned" for the controller's
 * decisions themselves -- its outputs are pinned by the dense-exponential
 * checks to within the requested tolerance).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- shallow-water model on the icosahedral grid ---------------- */
typedef struct {
    int n;                 /* number of cells N_g */
    double radius, omega, gravity, gamma_h, dt_e, nu;
    /* mesh (copied) */
    double *xyz;           /* n*3 unit vectors (cell centres = normals n_i) */
    int *deg, *nbr;        /* n, n*6 (ccw, pentagon slot 5 = self) */
    /* geometry derived here */
    double *area;          /* A_i (m^2) */
    double *len;           /* n*6 Voronoi edge length l_e (m) */
    double *dist;          /* n*6 centre distance d_e (m) */
    double *nrm;           /* n*6*3 unit outward edge normal n_{e,i} */
    double *tng;           /* n*6*3 unit edge tangent t_{e,i} = rhat_e x n_{e,i} */
    double *cor;           /* n Coriolis f_i = 2 Omega sin(lat_i) */
    double *work;          /* scratch, 16*n */
    double *hs;            /* n surface topography h_s (m); zero unless set */
} orc_swe;

int  orc_swe_init(orc_swe *m, int n, const double *xyz, const int *deg, const int *nbr,
                  const double *corners, double radius, double omega, double gravity,
                  double gamma_h, double dt_e);
void orc_swe_free(orc_swe *m);
/* h_s of the energy E = |u|^2/2 + g (h + h_s) in eq. sweqsinv (NULL: zero) */
void orc_swe_set_topography(orc_swe *m, const double *hs);

/* discrete operators (single field, length n) */
void orc_div(const orc_swe *m, const double *fx, const double *fy, const double *fz, double *out);
void orc_grad(const orc_swe *m, const double *psi, double *gx, double *gy, double *gz);
void orc_curl(const orc_swe *m, const double *ux, const double *uy, const double *uz, double *out);
void orc_lap(const orc_swe *m, const double *psi, double *out);

/* F(u), J(u)v, J(u)^T w ; vectors are [ux | uy | uz | h], length 4n */
void orc_rhs(const orc_swe *m, const double *u, double *f);
void orc_jv(const orc_swe *m, const double *u, const double *v, double *out);
void orc_jtv(const orc_swe *m, const double *u, const double *w, double *out);
/* K(a, b) = grad_u <a, J(u) b>, independent of u because F is quadratic */
void orc_ktv(const orc_swe *m, const double *a, const double *b, double *out);

/* Conserved quantities monitored in Sec. 6 (conservation paragraph), summed
 * over the cells with the cell areas: out[0] = mass sum A h, out[1] = total
 * energy sum A (h |u|^2 / 2 + g h^2 / 2 + g h h_s), out[2] = potential
 * enstrophy sum A (zeta + f)^2 / (2 h), zeta by the Stokes vorticity.  (The
 * paper prints the energy density as g h + |u|^2 / 2; the quantity the
 * continuous equations conserve is the one above.) */
void orc_diagnostics(const orc_swe *m, const double *u, double out[3]);

/* ---------------- small dense linear algebra ---------------- */
/* X = exp(A), A and X row-major KxK.  Returns the number of squarings. */
int  orc_expm(int K, const double *A, double *X);

/* ---------------- phipm_simul_iom2 ---------------- */
typedef void (*orc_matvec_fn)(void *ctx, const double *x, double *y);

enum { ORC_FREE = 0, ORC_RECORD = 1, ORC_REPLAY = 2 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENOTCONV = -4, ORC_ENAN = -5,
       ORC_ESCHED = -7 };

/* one attempt of the substep loop: the tau actually used, the Krylov size,
 * flag bit 0 = accepted, bit 1 = landed exactly on the output time */
typedef struct { double tau; int32_t m; int32_t flags; } orc_attempt;

typedef struct {
    orc_attempt *a;
    int len, cap, pos;
} orc_schedule;

/* What the solution of one accepted substep is made of: on [t, t + tau],
 *   y(t + s) = sum_{j<p} s^j/j! w_j + beta V_{m+1} c(s),
 * with c(s) the first m+1 entries of column m+p of exp(s Hhat'),
 * Hhat' = [[Hbar, e_1 e_1^T], [0, N_p]], Hbar = [[H_m, 0], [h e_m^T, 0]]. */
typedef struct {
    double t, tau, t_out; /* substep start, length, output time it heads for */
    int m;                /* Krylov size of the accepted attempt (0 when w_p = 0) */
    int out;              /* output index the substep lands on, -1 if none */
    double beta, hsub;    /* ||w_p|| and h_{m+1,m} (0 after a breakdown) */
    double *H;            /* m x m, row-major */
    double *V;            /* (m+1) x n: v_1 .. v_{m+1} (one zero vector when m = 0) */
    double *w;            /* p x n: w_0 .. w_{p-1} */
} orc_substep;

typedef struct {
    int n, p, len, cap;
    orc_substep *s;
} orc_phi_tape;

void orc_tape_free(orc_phi_tape *t);

typedef struct {
    double tol;            /* relative: Tol_abs = tol * max_l ||v_l|| */
    int m_init, m_max;
    double delta;          /* acceptance safety factor (1.4) */
    double gamma;          /* controller safety (0.8) */
    int max_attempts;
    int mode;              /* ORC_FREE / ORC_RECORD / ORC_REPLAY */
    orc_schedule *sched;   /* used in RECORD and REPLAY */
    orc_phi_tape *tape;    /* if set: every accepted substep is appended */
} orc_phi_opts;

typedef struct {
    int attempts, rejected, accepted, matvecs, expms, sum_m, max_m, last_m;
    int rec_matvecs;       /* products spent in the w_j recurrence */
} orc_phi_stats;

void orc_phi_default_opts(orc_phi_opts *o);

/* eq. cost (Sec. 4.3): estimated work of reaching the output time from t
 * with substeps tau and Krylov size m; remaining = t_out - t, n = problem
 * size, hnorm = ||tau Hhat||_1 of the augmented matrix at this tau.  The
 * controller changes tau iff C(tau_new, m) < C(tau, m_new). */
double orc_phi_cost(double tau, int m, int p, double remaining, double n, double hnorm);

/* Threads of the oracle's cell loops (OpenMP; default 1).  Only loops whose
 * iterations write disjoint outputs run in parallel; every sum keeps its
 * serial order, so results are bitwise the same for any thread count. */
void orc_set_threads(int nthreads);
int  orc_get_threads(void);

/* W_i = sum_l rho_i^l phi_l(rho_i A) v_l, i = 1..ns.  v[l] == NULL means the
 * zero vector.  *m_warm: in = starting Krylov size (<= 0: opts->m_init),
 * out = Krylov size of the last accepted attempt. */
int orc_phi_combo(int n, orc_matvec_fn A, void *actx, int p, const double *const *v,
                  int ns, const double *rho, double *const *w_out,
                  const orc_phi_opts *o, int *m_warm, orc_phi_stats *st);

/* dense-matrix convenience: A row-major n x n */
int orc_phi_combo_dense(int n, const double *A, int p, const double *const *v, int ns,
                        const double *rho, double *const *w_out, const orc_phi_opts *o,
                        int *m_warm, orc_phi_stats *st);

/* ---------------- adjoint of a phi-combination ---------------- */
/* acc += scale * K(a, b), K the derivative of <a, A(u) b> with respect to
 * whatever A depends on (acc's length is the caller's business) */
typedef void (*orc_kacc_fn)(void *ctx, const double *a, const double *b, double scale,
                            double *acc);

/* Cotangents of one phipm_simul_iom2 call from the tape of its forward
 * solve: vbar[l] (l = 0..p, NULL entries skipped) and kacc += int K(mu, y).
 * AT applies A^T.  p >= 1. */
int orc_phi_adjoint(int n, orc_matvec_fn AT, void *atctx, orc_kacc_fn K, void *kctx,
                    double *kacc, const orc_phi_tape *tape, int p, int ns, const double *rho,
                    const double *const *wbar, double *const *vbar, const orc_phi_opts *o,
                    orc_phi_stats *st);

/* dense A: forward (w_out) and adjoint (vbar, Abar = dL/dA, n x n) */
int orc_phi_vjp_dense(int n, const double *A, int p, const double *const *v, int ns,
                      const double *rho, const double *const *wbar, double *const *w_out,
                      double *const *vbar, double *Abar, const orc_phi_opts *o,
                      orc_phi_stats *fwd, orc_phi_stats *adj);

/* ---------------- exponential Rosenbrock schemes ---------------- */
enum { ORC_EXPRB42 = 0, ORC_PEXPRB43 = 1, ORC_EXPRB53 = 2, ORC_EPI3 = 3, ORC_EPI2 = 4,
       ORC_EXPRB42M = 5, ORC_EXPRB32 = 6 };

typedef void (*orc_rhs_fn)(void *ctx, const double *u, double *f);
typedef void (*orc_jv_fn)(void *ctx, const double *u, const double *v, double *out);

typedef struct {
    int n;
    orc_rhs_fn rhs;
    orc_jv_fn jv;
    void *ctx;
} orc_problem;

typedef struct {
    int m_warm[3];         /* warm-start Krylov size per call site */
    int have_prev;         /* epi3 history valid */
    double *u_prev, *f_prev;
    orc_phi_stats calls[3];
} orc_step_state;

int  orc_step_state_init(orc_step_state *s, int n);
void orc_step_state_free(orc_step_state *s);

int orc_step(const orc_problem *pb, int method, double *u, double dt, orc_step_state *s,
             const orc_phi_opts *o);

/* Vector-Jacobian product of one step (exprb42 only): ubar_n = (du_{n+1}/du_n)^T
 * ubar_np1, with the step recomputed under *o (replay its schedule to follow
 * the original forward).  adj: stats of the two adjoint calls (nullable). */
int orc_step_vjp(const orc_swe *m, int method, const double *u, double dt,
                 const double *ubar_np1, double *ubar_n, const orc_phi_opts *o,
                 orc_phi_stats *adj);

/* SWE problem wrapper usable as orc_problem ctx */
void orc_swe_problem(orc_swe *m, orc_problem *pb);

#ifdef __cplusplus
}
#endif
#endif
