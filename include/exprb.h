/*
 * exprb -- exponential Rosenbrock integration of the rotating shallow-water
 * equations on icosahedral geodesic grids, native to AMD MI355X (gfx950).
 *
 * C ABI of libexprb.so.  Plain pointers and sizes only.
 *
 * Conventions
 *  - A state or direction vector is FP64, length 4N, laid out as
 *    [u_x | u_y | u_z | h] with each block N cells long, in the cell order of
 *    the mesh passed to xrb_create (the state layout of Sec. 2, eq. dynu:
 *    Cartesian velocity components and fluid depth).
 *  - Vector arguments of the compute calls are DEVICE pointers owned by the
 *    caller; they must stay valid until the enqueued work has finished.
 *    Scalars, rho arrays and pointer arrays are HOST memory.
 *  - Work is enqueued on the context's HIP stream.  Calls return XRB_OK once
 *    the launches were accepted.  xrb_phi_combo and xrb_step synchronise the
 *    stream internally once per substep attempt (the host decides how many
 *    Krylov iterations to launch), so they return after their work is done.
 *  - A context is not thread-safe; use one context per stream.
 *  - On error the call returns a negative xrb_status and xrb_last_error()
 *    describes it.  Failures found on the device or by the HIP runtime (NaN,
 *    non-convergence, a failing runtime call) are returned by the call that
 *    finds them and are also latched: xrb_sync returns the first one since
 *    the previous xrb_sync.
 *  - The mesh is given to xrb_create as host arrays (xrb_mesh) rather than a
 *    file: the grids are generated in memory, and the caller keeps the choice
 *    of file format.
 */
#ifndef EXPRB_H
#define EXPRB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xrb_ctx xrb_ctx;

typedef enum {
    XRB_OK = 0,
    XRB_EINVAL = -1,   /* bad argument (size, pointer, rho order, p, mode) */
    XRB_ENOMEM = -2,   /* device or host allocation failed */
    XRB_EDEVICE = -3,  /* a HIP runtime call failed */
    XRB_ENOTCONV = -4, /* substep loop exceeded max_attempts or tau underflowed */
    XRB_ENAN = -5,     /* NaN/Inf met in a norm or in the error estimate */
    XRB_ESTATE = -6,   /* context state does not allow the call */
    XRB_ESCHED = -7    /* replay schedule exhausted or inconsistent */
} xrb_status;

/* The schemes of Sec. 3.3 plus the comparison and starting methods:
 * exprb42 (eq. 3.11), pexprb43 (eq. 3.12), exprb53 (eq. 3.13),
 * epi3 (eq. epi3, started by one EPI2 step), EPI2 = exponential
 * Rosenbrock-Euler (eq. 3.5), and EXPRB42M = exprb42 with its two
 * phi_1(.) v evaluations in one call: (i) rho = [3/4, 1], v_1 = v gives U2 and
 * phi_1(A) v; (ii) rho = [1] with only v_3 = 32/9 dt D2 (Sec. 4.4's mapping
 * of eq. 3.11 with the first two outputs shared).  The same method as
 * exprb42 in exact arithmetic; results differ at the Krylov tolerance. */
typedef enum {
    XRB_EXPRB42 = 0,
    XRB_PEXPRB43 = 1,
    XRB_EXPRB53 = 2,
    XRB_EPI3 = 3,
    XRB_EPI2 = 4,
    XRB_EXPRB42M = 5
} xrb_method;

/* Substep schedule handling of phi_combo: FREE = the device controller
 * decides; RECORD = as FREE, and every attempt (tau used, Krylov size,
 * accept/land flags) is appended to the context's schedule; REPLAY = the
 * attempts are taken from a schedule given with xrb_schedule_set instead of
 * the controller (bitwise-reproducible reruns). */
typedef enum { XRB_FREE = 0, XRB_RECORD = 1, XRB_REPLAY = 2 } xrb_sched_mode;

/* Icosahedral geodesic grid, unit sphere, HOST arrays (copied by xrb_create):
 *   xyz[3*i+k]        cell centre i (unit vector), k = x, y, z
 *   deg[i]            5 (pentagon) or 6
 *   nbr[6*i+s]        neighbours in counter-clockwise order seen from outside;
 *                     a pentagon's slot 5 holds i itself
 *   corners[18*i+3*s+k] Voronoi vertex shared by i, nbr[s], nbr[s+1 mod deg]
 * Cell geometry (areas, edge lengths, normals) is derived from these. */
typedef struct {
    int64_t n_cells;
    const double *xyz;
    const int32_t *deg;
    const int32_t *nbr;
    const double *corners;
} xrb_mesh;

/* Model and evaluator parameters.
 *   radius, omega, gravity       sphere radius (m), rotation rate (1/s), g (m/s^2)
 *   gamma_h, dt_e                hyperdissipation D_f = -nu L^2 with
 *                                nu = gamma_h dxbar^4 / dt_e, dxbar = sqrt(4 pi a^2 / N)
 *                                (eqs. swdis, niu; n_gamma = 4)
 *   tol                          phi_combo tolerance, relative to max_l ||v_l||_2
 *   m_init, m_max                first / largest Krylov size (m_max <= XRB_MMAX_LIMIT)
 *   delta, gamma                 acceptance safety factor (Alg. 1: 1.4) and
 *                                controller safety factor (0.8)
 *   max_attempts                 cap on substep attempts per phi_combo call
 *   lanes                        tuning: lanes per cell in the stencil kernels,
 *                                1, 2, 4 or 8, or 0 to choose from the grid size
 *                                (8 up to 16384 cells, else 2; with 0, batched
 *                                steps on grids up to 16384 cells use 2).  On
 *                                grids up to 16384 cells two and eight lanes
 *                                give the same bits; on larger ones two lanes
 *                                take the LDS-staged product, whose rounding
 *                                differs; 1 and 4 differ at the rounding level
 *                                (the order of the edge sums).  Results never
 *                                depend on the batch size. */
typedef struct {
    double radius, omega, gravity, gamma_h, dt_e;
    double tol;
    int32_t m_init, m_max;
    double delta, gamma;
    int32_t max_attempts;
    int32_t lanes;
} xrb_params;

#define XRB_MMAX_LIMIT 44
#define XRB_PMAX 4

typedef struct {
    int32_t attempts, rejected, accepted, matvecs, expms, sum_m, max_m, last_m, rec_matvecs;
} xrb_phi_stats;

/* Fill p with the defaults (a = 6.371e6 m, Omega = 7.292e-5 1/s,
 * g = 9.80616 m/s^2, gamma_h = 4e-4, dt_e = 240 s, tol = 1e-10, m_init = 1,
 * m_max = 40, delta = 1.4, gamma = 0.8, max_attempts = 10000, lanes = 0). */
xrb_status xrb_default_params(xrb_params *p);

/* Create a context on the current HIP device.  `stream` is a hipStream_t (NULL
 * = the default stream).  Allocates all device workspace (Krylov basis of
 * m_max+1 vectors plus stage vectors, about (m_max + 24) * 32 N bytes).
 * Errors: EINVAL (mesh inconsistent, m_max out of range), ENOMEM, EDEVICE. */
xrb_status xrb_create(const xrb_mesh *mesh, const xrb_params *params, void *stream,
                      xrb_ctx **out);
xrb_status xrb_destroy(xrb_ctx *ctx);
xrb_status xrb_set_stream(xrb_ctx *ctx, void *stream);
/* Wait for all work enqueued on the context's stream, then return the first
 * device-side failure (XRB_ENAN, XRB_ENOTCONV or XRB_EDEVICE) latched since
 * the previous xrb_sync and clear it; XRB_OK if there was none.  A failing
 * stream synchronisation itself returns XRB_EDEVICE. */
xrb_status xrb_sync(xrb_ctx *ctx);
const char *xrb_last_error(const xrb_ctx *ctx);
int64_t xrb_n_cells(const xrb_ctx *ctx);

/* The context's grid: *n_cells, and (each optional, NULL to skip) HOST
 * pointers to the cell centres xyz[3 n_cells] (unit vectors, the mesh's cell
 * order) and the cell areas area[n_cells] in m^2 (spherical polygon areas on
 * the sphere of params.radius, the A_i of the finite-volume operators of
 * Sec. 2).  The arrays belong to the context and stay valid until
 * xrb_destroy. */
xrb_status xrb_mesh_info(const xrb_ctx *ctx, int64_t *n_cells, const double **xyz,
                         const double **area);

/* f = F(u): the semi-discrete shallow-water right-hand side of eq. sweqsinv
 * (vector-invariant momentum with absolute vorticity eq. vort, flux-form
 * continuity; h_s = 0 unless set by xrb_set_topography) plus D_f = -nu L^2
 * on every variable (eq. swdis).
 * u, f: device, length 4N, must not alias. */
xrb_status xrb_rhs(xrb_ctx *ctx, const double *u, double *f);

/* jv = J(u) v with J = J_v + J_r + J_m of eqs. dynjs-dynjc (the Jacobian of
 * F, so the row-2 rotation signs follow from P_y = n_z u_x - n_x u_z).
 * Device vectors of length 4N; jv must not alias u or v. */
xrb_status xrb_jv(xrb_ctx *ctx, const double *u, const double *v, double *jv);

/* xrb_jv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same bits as xrb_jv, with its intermediates (the
 * cell-major copies of u and v, eta, the linearisation record, L v and the
 * product before its relayout, 200 bytes per cell) in a static device array
 * of 128 MiB that the library holds on every GPU it runs on until the
 * process ends.  The call allocates nothing; the context must exist
 * (xrb_create allocates).  Grids of more than 671 088 cells return
 * XRB_EINVAL before any work.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (two streams, two
 * contexts, two threads) race and must be serialised by the caller.
 * u, v, jv: device, length 4N; jv must not alias u or v. */
xrb_status xrb_jv_static(xrb_ctx *ctx, const double *u, const double *v, double *jv);

/* out = J(u)^T w, the Euclidean transpose of xrb_jv (the adjoint operator of
 * the linearised model; not in the paper, which has no adjoint).  Device
 * vectors of length 4N; out must not alias u or w.  The first call of any
 * adjoint entry point allocates the adjoint workspace (about
 * (2 m_max + 17) 32 N bytes). */
xrb_status xrb_jtv(xrb_ctx *ctx, const double *u, const double *w, double *out);

/* out = K(a, b) = grad_u <a, J(u) b>: the derivative of the Jacobian product
 * with respect to the linearisation state.  F is quadratic in u, so J is
 * affine in u and K does not depend on u: <d, K(a, b)> = <a, (J(d) - J(0)) b>.
 * Device vectors of length 4N; out must not alias a or b. */
xrb_status xrb_ktv(xrb_ctx *ctx, const double *a, const double *b, double *out);

/* Launch-shape autotuner: the launch shapes of the stencil kernels chosen
 * by measurement on this context's grid, in two stages.
 * 1. Lanes per cell: for each lane count 1, 2, 4, 8 it times one IOM2
 *    column's product (the Laplacian pass where that is separate, then the
 *    product with its dot epilogue; 3 warm-up and 20 timed launches on zero
 *    data, the fastest of 3 trials, HIP events) for a single state and for a
 *    batch of nm_batch members (1..256), and sets the context's lanes for
 *    single-state launches and for launches over many cells to the pair that
 *    minimises the sum of the two times relative to each one's best, among
 *    the pairs that keep batched members bitwise equal to single runs (the
 *    same count, or two and eight on grids up to 16384 cells, which carry no
 *    chunk tables); the current pair is kept unless that one is more than
 *    3 % better.  Overrides xrb_params.lanes.
 * 2. Block shapes, at the chosen lanes (none of them changes a result bit):
 *    where a gather product sums per-cell terms in cell order (grids up to
 *    65536 cells, not two lanes with chunk tables), the threads per product
 *    block (the one-pass size, half of it, 256 and 512), separately for
 *    single states and batches, and the threads per Laplacian block (64,
 *    128, 256); with the LDS-staged kernels (two lanes, grids above 16384
 *    cells), the blocks of the Laplacian launch (512, 1024, 2048, at most
 *    one per chunk).  The built-in rule is kept unless a candidate is more
 *    than 3 % faster.
 * Every batched launch covers all members (the member-minor launch order was
 * measured and lost).  Synchronises the stream; allocates 8 nm_batch vectors
 * for its duration.  out (host): the timings in microseconds per launch and
 * the choices (0 = the built-in rule). */
typedef struct {
    double single_us[4];   /* lanes 1, 2, 4, 8: one state */
    double batch_us[4];    /* lanes 1, 2, 4, 8: nm_batch members in one launch */
    int32_t lanes;         /* chosen for single-state launches */
    int32_t lanes_batch;   /* chosen for launches over more than 200000 cells in all */
    int32_t nm_batch;
    int32_t jv_cand[4];    /* product threads tried (0: unused slot) */
    double jv_single_us[4], jv_batch_us[4];
    int32_t jv_block, jv_block_batch;
    int32_t lap_cand[3];   /* Laplacian threads (gather form) or blocks (LDS form) tried */
    double lap_us[3];
    int32_t lap_block, lap_grid;
} xrb_tune_result;
xrb_status xrb_autotune(xrb_ctx *ctx, int nm_batch, xrb_tune_result *out);

/* Surface topography h_s of the model (the h_s in the energy
 * E = |u|^2 / 2 + g (h + h_s) of eq. sweqsinv, Sec. 2): hs is a HOST array of
 * n_cells heights in metres, in the mesh's cell order, copied to the device
 * (NULL restores the flat default).  Only F(u) depends on it (J does not:
 * h_s is constant in time).  Synchronises the context's stream first.
 * XRB_EINVAL for non-finite values, XRB_ENOMEM if the copy cannot be
 * allocated. */
xrb_status xrb_set_topography(xrb_ctx *ctx, const double *hs);

/* Conserved quantities of the state u (the three the conservation
 * paragraph of Sec. 6 monitors), summed over the cells with their areas A:
 *   out3[0] = mass                sum A h,
 *   out3[1] = total energy        sum A (h |u|^2 / 2 + g h^2 / 2 + g h h_s),
 *   out3[2] = potential enstrophy sum A (zeta + f)^2 / (2 h),
 * zeta the Stokes vorticity of the grid and f = 2 Omega z.  (The paper
 * prints the energy density as g h + |u|^2 / 2; the total energy the
 * equations conserve without topography is the one above.)  u: device,
 * [u_x | u_y | u_z | h], h > 0; out3: host, 3 doubles.  Synchronises the
 * context's stream; the sums are in a fixed order (bitwise reproducible).
 * XRB_EINVAL on null pointers. */
xrb_status xrb_diagnostics(xrb_ctx *ctx, const double *u, double *out3);

/* Vector-Jacobian product of one step (method XRB_EXPRB42 only):
 * ubar_n = (d u_{n+1} / d u_n)^T ubar_np1 for u_{n+1} = step(u_n, dt).
 * The step is recomputed on the device, following `sched` (host, sched_len
 * entries of (tau, m, flags) as xrb_schedule_get returns them for that one
 * step) or, with sched = NULL, the free controller from a cold start.  The
 * reverse sweep is the continuous adjoint of each phi-combination on the
 * recomputed substeps: a Krylov space of (dt J)^T per substep (IOM2, the
 * forward's tau, Krylov size grown from the forward's until the correction
 * estimate passes, at most m_max), the adjoint moments from one augmented
 * exponential, and the A-term int K(mu, y) dt exactly through a Van Loan
 * block exponential; then the scheme's chain rule.
 *   u         device, the state u_n (not modified)
 *   ubar_np1  device, the cotangent of u_{n+1}; ubar_n device output (may
 *             alias ubar_np1, not u)
 *   stats     optional host [2]: statistics of the two adjoint calls
 *             (attempts = exponential tests, rejected = substeps taken at
 *             m_max without passing the test); non-NULL forces a sync.
 * The substeps of the recomputed forward are stored on the device (about
 * (m_max + 5) 32 N bytes per accepted substep, kept for later calls). */
xrb_status xrb_step_vjp(xrb_ctx *ctx, xrb_method method, const double *u, double dt,
                        const double *sched, int sched_len, const double *ubar_np1,
                        double *ubar_n, xrb_phi_stats *stats);

/* W_i = sum_{l=0}^p rho_i^l phi_l(rho_i dt J(u)) v_l, i = 1..ns
 * (phipm_simul_iom2, Alg. 1 of Sec. 4.3; the multi-output form of
 * eq. exp_multistage with the rho^l weights that make W_i the solution of
 * eq. 3.15 at t = rho_i).
 *   dt     scaling of the Jacobian (A = dt J(u))
 *   u      device, linearisation state
 *   p      0 <= p <= XRB_PMAX
 *   v      host array of p+1 device pointers; NULL = zero vector (enables the
 *          zero-skip of Sec. 4.3)
 *   ns     1 <= ns <= 8; rho host array, 0 < rho_1 < ... < rho_ns <= 1
 *   w_out  host array of ns device pointers, must not alias u or any v
 *   stats  optional host output
 * Substeps follow the context's schedule mode.  Each call starts at Krylov
 * size m_init (the scheme driver xrb_step keeps per-call-site warm starts).
 * Errors: EINVAL (sizes, rho order, aliasing that can be seen), ENOTCONV,
 * ENAN, ESCHED (replay schedule exhausted), EDEVICE. */
xrb_status xrb_phi_combo(xrb_ctx *ctx, double dt, const double *u, int p,
                         const double *const *v, int ns, const double *rho,
                         double *const *w_out, xrb_phi_stats *stats);

/* One step u <- u_{n+1} of `method` with step size dt (device u, in place),
 * through the phi_combo call mapping of Sec. 4.4 with A = dt J(u_n),
 * v = dt F(u_n).  Each scheme call site keeps its own Krylov warm start;
 * epi3 keeps u_{n-1} and F(u_{n-1}) in the context (the first epi3 step, or
 * the first after xrb_reset_history, is an EPI2 step). */
xrb_status xrb_step(xrb_ctx *ctx, xrb_method method, double *u, double dt);

/* One step of `method` for nm independent ensemble members in one batched
 * sequence of launches: every kernel covers all members, and the members'
 * substep controllers (Alg. 1) advance in lockstep rounds, each with its own
 * step size, Krylov sizes and substeps; a member that needs fewer Krylov
 * columns or substeps skips the launches of the others.
 *   U      device, nm x 4N, member-major (member k at U + 4N k), in place
 *   dt     host [nm], positive step sizes
 *   stats  optional host [nm][3] per-member, per-call-site statistics
 * The ensemble keeps its own per-member warm starts and epi3 history; the
 * first call with a given nm allocates an nm-member workspace (about
 * nm (m_max + 35) 32 N bytes), a call with another nm replaces it.  Results
 * equal those of xrb_step on each member alone (same kernels, same
 * reduction order).  In RECORD and REPLAY mode each member has a schedule
 * of its own (xrb_schedule_get_member / xrb_schedule_set_member). */
xrb_status xrb_step_batch(xrb_ctx *ctx, xrb_method method, int nm, double *U, const double *dt,
                          xrb_phi_stats *stats);

/* The batched step above as one HIP graph (the ensemble's whole launch
 * sequence, not in the paper): with the context in REPLAY mode, the host
 * knows every substep decision of every member from its schedule
 * (xrb_schedule_set_member), so it walks all attempt rounds without waiting
 * for the device's decision records or synchronising, while the stream is
 * captured; every host-to-device upload of the rounds (plans, controller
 * arguments, step sizes) is staged in a pinned arena that the context keeps.
 * xrb_step_batch_capture records that step for U and dt (it consumes the
 * members' schedule entries as xrb_step_batch would, and runs nothing);
 * xrb_graph_launch runs it, waits, and reports a device failure from the
 * members' last decisions.  A launch gives the bits of the same replayed
 * xrb_step_batch.  U, dt and the context's ensemble workspace are baked into
 * the graph: relaunches step whatever U then holds with the same schedule,
 * and a new capture, a batched call with another nm, or xrb_destroy drops
 * the graph.  Every member's inputs are taken as nonzero (a member at rest
 * needs the eager call).  Errors: EINVAL (not in REPLAY mode, event
 * profiling on, the null stream, nothing captured), ESCHED (a schedule runs
 * out), ENOMEM, EDEVICE. */
xrb_status xrb_step_batch_capture(xrb_ctx *ctx, xrb_method method, int nm, double *U,
                                  const double *dt);
xrb_status xrb_graph_launch(xrb_ctx *ctx);

/* A general exponential Rosenbrock scheme (eq. 3.10: internal stages U_ni
 * and weights built from phi_k functions of c_i dt J_n, whose stiff order
 * conditions Table 1 lists) written as the sequence of phi-combination
 * calls of Sec. 4.4.  With A = dt J(u_n), v = dt F(u_n) and the nonlinear
 * remainders D_i = F(U_i) - F(u_n) - J(u_n)(U_i - u_n) (eq. Dni):
 *   call c = 0..ncalls-1, in order:
 *     v_l = vc[c][l][0] v + sum_s vc[c][l][1+s] dt D_{s+2}   (l = 1..p[c]; v_0 = 0),
 *     outputs W_{c,o} = sum_l rho[c][o]^l phi_l(rho[c][o] A) v_l, o < ns[c]
 *     (0 < rho[c][0] < rho[c][1] <= 1; the rho^l weights as in xrb_phi_combo);
 *   after call c, each stage s with stage_call[s] == c:
 *     U_{s+2} = u_n + sum_{c' <= c, o} uc[s][c'][o] W_{c',o}, then D_{s+2};
 *   u_{n+1} = u_n + sum_{c, o} un1[c][o] W_{c,o}.
 * A v_l may use only remainders of stages defined before call c.  Call site
 * c keeps its own Krylov warm start, as in xrb_step.  The built-in schemes
 * written this way give the same bits as xrb_step (the same vector
 * combinations in the same order).  Limits: 3 calls of 2 outputs, 2
 * internal stages, p[c] <= XRB_PMAX, at most 5 nonzero output terms in a
 * stage or in u_{n+1}.  Errors: EINVAL (limits, rho order, a remainder used
 * before its stage), then as xrb_step. */
#define XRB_TAB_CALLS 3
#define XRB_TAB_OUT 2
#define XRB_TAB_STAGES 2
typedef struct {
    int ncalls;
    int p[XRB_TAB_CALLS];
    int ns[XRB_TAB_CALLS];
    double rho[XRB_TAB_CALLS][XRB_TAB_OUT];
    double vc[XRB_TAB_CALLS][XRB_PMAX + 1][1 + XRB_TAB_STAGES];
    int nstages;
    int stage_call[XRB_TAB_STAGES];
    double uc[XRB_TAB_STAGES][XRB_TAB_CALLS][XRB_TAB_OUT];
    double un1[XRB_TAB_CALLS][XRB_TAB_OUT];
} xrb_tableau;
xrb_status xrb_step_tableau(xrb_ctx *ctx, const xrb_tableau *tab, double *u, double dt);

/* Per-call-site statistics of the last xrb_step (3 entries). */
xrb_status xrb_step_stats(const xrb_ctx *ctx, xrb_phi_stats *out3);

/* Forget warm starts, epi3 history and the recorded schedule. */
xrb_status xrb_reset_history(xrb_ctx *ctx);

/* Schedule control.  Entries are host triples (tau, m, flags) with flags
 * bit 0 = accepted, bit 1 = landed on an output time.  xrb_schedule_set
 * copies `len` entries and rewinds the replay cursor; xrb_schedule_get copies
 * up to `cap` recorded entries and reports the total in *len. */
xrb_status xrb_schedule_mode(xrb_ctx *ctx, int mode);
xrb_status xrb_schedule_set(xrb_ctx *ctx, const double *entries, int len);
xrb_status xrb_schedule_get(const xrb_ctx *ctx, double *entries, int cap, int *len);
/* The same for member k of the batched steps (xrb_step_batch): every member
 * records into, or replays from, a schedule of its own.  A batched step in
 * REPLAY mode fails with XRB_ESCHED if a member has no schedule or runs out
 * of entries.  xrb_schedule_mode rewinds every member's replay cursor and
 * xrb_reset_history forgets the member schedules. */
xrb_status xrb_schedule_set_member(xrb_ctx *ctx, int k, const double *entries, int len);
xrb_status xrb_schedule_get_member(const xrb_ctx *ctx, int k, double *entries, int cap,
                                   int *len);

/* Optional per-kernel timing.  xrb_profile(ctx, N) with N >= 1 zeroes the
 * counters and brackets every N-th launch of each kernel below (made by
 * xrb_phi_combo / xrb_step) with a pair of HIP events on the context's
 * stream; N = 1 times every launch, a larger N samples and keeps the event
 * overhead out of most launches.  Times are collected at the
 * synchronisation points the calls already have.  xrb_profile(ctx, 0)
 * disables.  Kernel ids: */
enum {
    XRB_K_JV_IOM2 = 0,   /* Jacobian product fused with the IOM2 dots   */
    XRB_K_LAP = 1,       /* one-ring Laplacian pass (L x)               */
    XRB_K_IOM2_UPD = 2,  /* IOM2 two-term update + norm                 */
    XRB_K_CTL = 3,       /* augmented exponential + controller          */
    XRB_K_COMBINE = 4,   /* substep combination y_{k+1}                 */
    XRB_K_JV_OTHER = 5,  /* Jacobian products of the w_j recurrence/stages */
    XRB_K_RHS = 6,       /* right-hand side F(u)                        */
    XRB_K_VEC = 7,       /* linear combinations, norms                  */
    XRB_K_UPD_LAP = 8,   /* IOM2 update fused with the next column's L x
                            (grids above 16384 cells)                   */
    XRB_K_COUNT = 9
};
xrb_status xrb_profile(xrb_ctx *ctx, int enable);
/* Since the last xrb_profile(ctx, N >= 1): device milliseconds summed over
 * the timed launches of kernel `kernel`, the number of timed launches, and
 * the number of all launches of that kernel. */
xrb_status xrb_profile_get(const xrb_ctx *ctx, int kernel, double *timed_ms, int64_t *timed,
                           int64_t *launches);
/* What one event pair adds to a timed launch: `reps` launches of a one-wave
 * kernel that runs 20 us, each between its own pair of events on the
 * context's stream, minus the same launches back to back between one pair,
 * per launch, in microseconds (*us; reps of 200 take about 8 ms).  Subtracting it from xrb_profile's per-launch averages
 * leaves the kernel's own duration plus the gap between consecutive
 * launches.  Synchronises the stream; reps in 1..100000. */
xrb_status xrb_profile_overhead(xrb_ctx *ctx, int reps, double *us);

#ifdef __cplusplus
}
#endif
#endif
