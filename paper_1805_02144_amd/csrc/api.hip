// C ABI of libexprb: context, phipm_simul_iom2 driver (Alg. 1) and the
// exponential Rosenbrock scheme drivers (Sec. 4.4).
//
// The substep loop of Alg. 1 runs on the host only as a launcher: every
// arithmetic step (w_j recurrence, IOM2, augmented exponential, controller,
// substep update) is a device kernel; the host reads back one small decision
// record per attempt to know how many Krylov columns the next attempt needs.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "reduce.h"
#include "xrb_internal.h"

using namespace xrb;

struct SchedEntry {
    double tau;
    int32_t m;
    int32_t flags;
};

struct xrb_ctx {
    xrb_params prm{};
    int n = 0, n4 = 0;
    hipStream_t stream = nullptr;
    DevMesh M{};
    void *geo_mem = nullptr;
    double *V = nullptr;        // (m_max+1) raw basis vectors
    double *W = nullptr;        // w_1..w_{p-1}
    double *y = nullptr;
    double *lap = nullptr;      // L x scratch
    double *eta = nullptr;      // V.u + f at the current linearisation point
    double *stage = nullptr;    // 16 stage vectors of the schemes
    double *dot_parts = nullptr;   // IOM2 dot partials (2 per block)
    double *nrm_parts = nullptr;   // norm partials, two buffers: column j uses buffer j % 2
    double *v_parts = nullptr;     // norm partials of the phi_combo inputs
    double *vnorm2 = nullptr;
    PhiCtl *ctl = nullptr;
    Decision *dec_host = nullptr;
    double *vn_host = nullptr;
    std::string err;
    int mode = XRB_FREE;
    std::vector<SchedEntry> sched;
    size_t sched_pos = 0;
    int m_warm[3] = {0, 0, 0};
    int have_prev = 0;
    xrb_phi_stats last_stats[3]{};
    // optional per-kernel event timing
    struct Pending {
        int id;
        hipEvent_t a, b;
    };
    int prof_every = 0;            // 0 = off, N = time every N-th launch of each kernel
    int64_t prof_seen[XRB_K_COUNT] = {};
    std::vector<hipEvent_t> ev_free;
    std::vector<Pending> ev_pend;
    double prof_ms[XRB_K_COUNT] = {};
    int64_t prof_n[XRB_K_COUNT] = {};

    double *sv(int k) { return stage + (size_t)k * n4; }
};

namespace {

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);             \
            return XRB_EDEVICE;                                                       \
        }                                                                             \
    } while (0)

int fail(xrb_ctx *ctx, int code, const char *msg) {
    if (ctx) ctx->err = msg;
    return code;
}

hipEvent_t ev_get(xrb_ctx *ctx) {
    if (!ctx->ev_free.empty()) {
        hipEvent_t e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket a launch with events when profiling is on.
template <class F>
void timed(xrb_ctx *ctx, int id, F &&launch) {
    if (ctx->prof_every <= 0 || (ctx->prof_seen[id]++ % ctx->prof_every) != 0) {
        launch();
        return;
    }
    hipEvent_t a = ev_get(ctx), b = ev_get(ctx);
    if (!a || !b) {
        launch();
        return;
    }
    (void)hipEventRecord(a, ctx->stream);
    launch();
    (void)hipEventRecord(b, ctx->stream);
    ctx->ev_pend.push_back({id, a, b});
}

// Collect finished event pairs (called after a stream synchronisation).
void prof_drain(xrb_ctx *ctx) {
    for (auto &p : ctx->ev_pend) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->prof_ms[p.id] += ms;
            ctx->prof_n[p.id] += 1;
        }
        ctx->ev_free.push_back(p.a);
        ctx->ev_free.push_back(p.b);
    }
    ctx->ev_pend.clear();
}

// stage slots used by xrb_step
enum { S_FN, S_V, S_W1, S_W2, S_X1, S_X2, S_U2, S_U3, S_D2, S_D3, S_A3, S_A4, S_T1, S_T2,
       S_UPREV, S_FPREV, S_COUNT };

// J(u) x into out (kernel chain: L x, then the fused product); eta must hold V.u + f
void jv_plain(xrb_ctx *ctx, const double *u, const double *x, double *out, double dt) {
    timed(ctx, XRB_K_LAP, [&] { launch_lap4(ctx->M, x, ctx->lap, ctx->stream); });
    JvArgs a;
    a.u = u;
    a.eta = ctx->eta;
    a.x = x;
    a.lx = ctx->lap;
    a.dt = dt;
    a.out = out;
    timed(ctx, XRB_K_JV_OTHER, [&] { launch_jv(ctx->M, a, kEpiNone, ctx->stream); });
}

void rhs_plain(xrb_ctx *ctx, const double *u, double *f) {
    timed(ctx, XRB_K_LAP, [&] { launch_lap4(ctx->M, u, ctx->lap, ctx->stream); });
    timed(ctx, XRB_K_RHS, [&] { launch_rhs(ctx->M, u, ctx->lap, f, ctx->stream); });
}

void lincomb(xrb_ctx *ctx, double *out, std::initializer_list<const double *> vs,
             std::initializer_list<double> cs) {
    const double *vv[6];
    double cc[6];
    int k = 0;
    auto ci = cs.begin();
    for (auto v : vs) {
        vv[k] = v;
        cc[k] = *ci++;
        ++k;
    }
    timed(ctx, XRB_K_VEC, [&] { launch_lincomb(ctx->n4, out, k, vv, cc, ctx->stream); });
}

// phipm_simul_iom2 with eta = V.u + f already computed for u.
int phi_run(xrb_ctx *ctx, double dt, const double *u, int p, const double *const *v, int ns,
            const double *rho, double *const *w_out, int m_start, int *m_last,
            xrb_phi_stats *st_out) {
    xrb_phi_stats st{};
    const int n4 = ctx->n4;
    const hipStream_t s = ctx->stream;
    const xrb_params &P = ctx->prm;
    if (p < 0 || p > kPmax || ns < 1 || ns > 8 || !rho || !w_out || !v)
        return fail(ctx, XRB_EINVAL, "phi_combo: bad p, ns or null array");
    for (int i = 0; i < ns; ++i) {
        if (!(rho[i] > 0.0) || rho[i] > 1.0 || (i > 0 && !(rho[i] > rho[i - 1])))
            return fail(ctx, XRB_EINVAL, "phi_combo: rho must increase within (0, 1]");
        if (!w_out[i]) return fail(ctx, XRB_EINVAL, "phi_combo: null output");
        for (int l = 0; l <= p; ++l)
            if (v[l] && v[l] == w_out[i]) return fail(ctx, XRB_EINVAL, "phi_combo: output aliases input");
    }
    // scale = max_l ||v_l||; all-zero inputs give W = 0 exactly
    const int n = ctx->n;
    int np_r0 = 0, np_dot = 0, np_upd = 0;   // partial counts of the last producers
    const double *vl[kPmax + 1];
    int nv = 0;
    for (int l = 0; l <= p; ++l)
        if (v[l]) vl[nv++] = v[l];
    int m = m_start > 0 ? m_start : P.m_init;
    m = std::min(std::max(m, 1), P.m_max);
    int npv = 0;
    if (nv > 0) timed(ctx, XRB_K_VEC, [&] { npv = launch_norms(n, nv, vl, ctx->v_parts, s); });
    launch_phi_init(ctx->ctl, m, rho[0], P.tol, ctx->v_parts, npv, nv, ctx->vnorm2, s);
    HIPCHK(hipMemcpyAsync(ctx->vn_host, ctx->vnorm2, sizeof(double) * (kPmax + 1),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    prof_drain(ctx);
    double smax = 0.0;
    for (int k = 0; k < nv; ++k) {
        if (ctx->vn_host[k] != ctx->vn_host[k]) return fail(ctx, XRB_ENAN, "phi_combo: NaN input");
        smax = std::max(smax, ctx->vn_host[k]);
    }
    if (smax == 0.0) {
        for (int i = 0; i < ns; ++i) HIPCHK(hipMemsetAsync(w_out[i], 0, sizeof(double) * n4, s));
        if (st_out) *st_out = st;
        return XRB_OK;
    }
    int y_zero = 1;
    if (v[0]) {
        HIPCHK(hipMemcpyAsync(ctx->y, v[0], sizeof(double) * n4, hipMemcpyDeviceToDevice, s));
        y_zero = 0;
    }
    int wzero[kPmax + 1];
    const double *wptr[kPmax + 1];
    auto nrm_buf = [&](int col) { return ctx->nrm_parts + (size_t)(col & 1) * kRedBlocks; };
    bool point_ready = false;
    int built = 0, wp_zero = 0;

    for (int io = 0; io < ns; ++io) {
        launch_set_tout(ctx->ctl, rho[io], s);
        bool reached = false;
        while (!reached) {
            if (st.attempts >= P.max_attempts) return fail(ctx, XRB_ENOTCONV, "phi_combo: attempt cap");
            st.attempts++;
            ReplayIn rep{};
            if (ctx->mode == XRB_REPLAY) {
                if (ctx->sched_pos >= ctx->sched.size())
                    return fail(ctx, XRB_ESCHED, "phi_combo: replay schedule exhausted");
                const SchedEntry &e = ctx->sched[ctx->sched_pos++];
                if (e.m < 1 || e.m > P.m_max) return fail(ctx, XRB_ESCHED, "phi_combo: bad replay m");
                rep.tau = e.tau;
                rep.m = e.m;
                rep.flags = e.flags;
                rep.active = 1;
                m = e.m;
            }
            if (!point_ready) {
                // step 1: w_j recurrence (eq. 3.18) with the zero-skip of Sec. 4.3
                wzero[0] = y_zero;
                wptr[0] = ctx->y;
                for (int j = 1; j <= p; ++j) {
                    double *dst = (j == p) ? ctx->V : ctx->W + (size_t)(j - 1) * n4;
                    JvArgs a;
                    for (int l = 0; l <= p - j; ++l) {
                        if (!v[j + l] || (l > 0 && st.accepted == 0)) continue;
                        a.axv[a.naxpy] = v[j + l];
                        a.axc[a.naxpy] = &ctx->ctl->rec_coef[l];
                        a.naxpy++;
                    }
                    const int epi = (j == p) ? kEpiNorm : kEpiNone;
                    if (!wzero[j - 1]) {
                        timed(ctx, XRB_K_LAP, [&] { launch_lap4(ctx->M, wptr[j - 1], ctx->lap, s); });
                        a.u = u;
                        a.eta = ctx->eta;
                        a.x = wptr[j - 1];
                        a.lx = ctx->lap;
                        a.dt = dt;
                        a.out = dst;
                        a.ctl = ctx->ctl;
                        a.nrm_out = ctx->nrm_parts;
                        timed(ctx, XRB_K_JV_OTHER, [&] {
                            const int g = launch_jv(ctx->M, a, epi, s);
                            if (j == p) np_r0 = g;
                        });
                        st.matvecs++;
                        st.rec_matvecs++;
                        wzero[j] = 0;
                    } else if (a.naxpy > 0) {
                        timed(ctx, XRB_K_VEC, [&] {
                            const int g = launch_lincomb_dev(n, dst, a.naxpy, a.axv, a.axc,
                                                             j == p ? ctx->nrm_parts : nullptr, s);
                            if (j == p) np_r0 = g;
                        });
                        wzero[j] = 0;
                    } else {
                        wzero[j] = 1;
                    }
                    wptr[j] = dst;
                }
                wp_zero = wzero[p];
                if (p == 0) {
                    // phi_0 only: the basis starts from y itself
                    if (!y_zero) {
                        const double *one[1] = {ctx->y};
                        const double *cf[1] = {&ctx->ctl->rec_coef[0]};
                        np_r0 = launch_lincomb_dev(n, ctx->V, 1, one, cf, ctx->nrm_parts, s);
                    }
                    wp_zero = y_zero;
                }
                built = 0;
                point_ready = true;
            }
            // step 2(i): IOM2 columns up to m
            if (!wp_zero) {
                for (int j = built; j < m; ++j) {
                    double *rj = ctx->V + (size_t)j * n4;
                    double *rn = ctx->V + (size_t)(j + 1) * n4;
                    const double *rm = j > 0 ? ctx->V + (size_t)(j - 1) * n4 : nullptr;
                    timed(ctx, XRB_K_LAP, [&] { launch_lap4(ctx->M, rj, ctx->lap, s); });
                    JvArgs a;
                    a.u = u;
                    a.eta = ctx->eta;
                    a.x = rj;
                    a.lx = ctx->lap;
                    a.dt = dt;
                    a.out = rn;
                    a.j = j;
                    a.rjm1 = rm;
                    a.ctl = ctx->ctl;
                    a.dot_out = ctx->dot_parts;
                    timed(ctx, XRB_K_JV_IOM2, [&] { np_dot = launch_jv(ctx->M, a, kEpiIom2, s); });
                    const int np_in = (j == 0) ? np_r0 : np_upd;
                    timed(ctx, XRB_K_IOM2_UPD, [&] {
                        np_upd = launch_iom2_update(n, j, rn, rj, rm, ctx->ctl, nrm_buf(j), np_in,
                                                    ctx->dot_parts, np_dot, nrm_buf(j + 1), s);
                    });
                    st.matvecs++;
                }
                built = std::max(built, m);
            }
            // steps 2(ii)-6 on the device
            CtlArgs ca;
            ca.m = m;
            ca.p = p;
            ca.mode = ctx->mode;
            ca.m_max = P.m_max;
            ca.wp_zero = wp_zero;
            ca.built = built;
            ca.nrm_in = nrm_buf(built);
            ca.n_nrm_in = np_upd;
            ca.n4 = (double)n4;
            ca.delta = P.delta;
            ca.gamma = P.gamma;
            ca.rep = rep;
            timed(ctx, XRB_K_CTL, [&] { launch_controller(ctx->ctl, ca, s); });
            HIPCHK(hipMemcpyAsync(ctx->dec_host, &ctx->ctl->dec, sizeof(Decision),
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            prof_drain(ctx);
            const Decision d = *ctx->dec_host;
            if (d.status == XRB_ENAN) return fail(ctx, XRB_ENAN, "phi_combo: NaN in Krylov process");
            if (d.status != 0) return fail(ctx, d.status, "phi_combo: device error");
            if (!(d.tau_u >= 1e-12 * rho[ns - 1]))
                return fail(ctx, XRB_ENOTCONV, "phi_combo: substep underflow");
            if (d.m_eff > 0) st.expms++;
            st.sum_m += m;
            st.max_m = std::max(st.max_m, m);
            if (ctx->mode == XRB_RECORD)
                ctx->sched.push_back({d.tau_u, m, (d.accept ? 1 : 0) | (d.lands ? 2 : 0)});
            if (d.accept) {
                timed(ctx, XRB_K_COMBINE, [&] {
                    launch_combine(n4, ctx->y, p, wptr, wzero, ctx->V, d.m_eff, d.m_eff > 0 ? 1 : 0,
                                   ctx->ctl, s);
                });
                st.accepted++;
                st.last_m = m;
                y_zero = 0;
                point_ready = false;
            } else {
                st.rejected++;
            }
            if (ctx->mode != XRB_REPLAY) m = d.m_next;
            reached = d.reached != 0;
        }
        HIPCHK(hipMemcpyAsync(w_out[io], ctx->y, sizeof(double) * n4, hipMemcpyDeviceToDevice, s));
    }
    if (m_last) *m_last = st.last_m;
    if (st_out) *st_out = st;
    return XRB_OK;
}

int free_all(xrb_ctx *ctx) {
    prof_drain(ctx);
    for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
    ctx->ev_free.clear();
    void *dev[] = {ctx->geo_mem, ctx->V, ctx->W, ctx->y, ctx->lap, ctx->eta, ctx->stage,
                   ctx->dot_parts, ctx->nrm_parts, ctx->v_parts, ctx->vnorm2, ctx->ctl};
    int rc = XRB_OK;
    for (void *p : dev)
        if (p && hipFree(p) != hipSuccess) rc = XRB_EDEVICE;
    if (ctx->dec_host && hipHostFree(ctx->dec_host) != hipSuccess) rc = XRB_EDEVICE;
    if (ctx->vn_host && hipHostFree(ctx->vn_host) != hipSuccess) rc = XRB_EDEVICE;
    return rc;
}

}  // namespace

extern "C" {

xrb_status xrb_default_params(xrb_params *p) {
    if (!p) return XRB_EINVAL;
    p->radius = 6.371e6;
    p->omega = 7.292e-5;
    p->gravity = 9.80616;
    p->gamma_h = 4e-4;
    p->dt_e = 240.0;
    p->tol = 1e-10;
    p->m_init = 1;
    p->m_max = 40;
    p->delta = 1.4;
    p->gamma = 0.8;
    p->max_attempts = 10000;
    return XRB_OK;
}

xrb_status xrb_create(const xrb_mesh *mesh, const xrb_params *params, void *stream,
                      xrb_ctx **out) {
    if (!mesh || !params || !out) return XRB_EINVAL;
    *out = nullptr;
    if (params->m_max < 1 || params->m_max > kMmax || params->m_init < 1 || !(params->tol > 0.0) ||
        params->max_attempts < 1 || !(params->radius > 0.0) || !(params->dt_e > 0.0))
        return XRB_EINVAL;
    xrb_ctx *ctx = new (std::nothrow) xrb_ctx();
    if (!ctx) return XRB_ENOMEM;
    ctx->prm = *params;
    ctx->stream = (hipStream_t)stream;
    HostGeometry geo;
    int rc = build_geometry(*mesh, *params, geo, ctx->err);
    if (rc) {
        delete ctx;
        return (xrb_status)rc;
    }
    const int n = geo.n;
    ctx->n = n;
    ctx->n4 = 4 * n;
    const size_t nd = (size_t)n;
    // geometry in one allocation: 7 x [6][n] weights, 4 x [n] cell fields, [6][n] int32
    const size_t dbl = 7 * 6 * nd + 4 * nd;
    const size_t bytes = dbl * sizeof(double) + 6 * nd * sizeof(int32_t);
    auto ck = [&](hipError_t e) {
        if (e != hipSuccess && rc == 0) {
            ctx->err = hipGetErrorString(e);
            rc = XRB_ENOMEM;
        }
    };
    ck(hipMalloc(&ctx->geo_mem, bytes));
    const size_t n4 = 4 * nd;
    ck(hipMalloc((void **)&ctx->V, sizeof(double) * n4 * (params->m_max + 1)));
    ck(hipMalloc((void **)&ctx->W, sizeof(double) * n4 * kPmax));
    ck(hipMalloc((void **)&ctx->y, sizeof(double) * n4));
    ck(hipMalloc((void **)&ctx->lap, sizeof(double) * n4));
    ck(hipMalloc((void **)&ctx->eta, sizeof(double) * nd));
    ck(hipMalloc((void **)&ctx->stage, sizeof(double) * n4 * S_COUNT));
    ck(hipMalloc((void **)&ctx->dot_parts, sizeof(double) * 2 * kRedBlocks));
    ck(hipMalloc((void **)&ctx->nrm_parts, sizeof(double) * 2 * kRedBlocks));
    ck(hipMalloc((void **)&ctx->v_parts, sizeof(double) * (kPmax + 1) * kRedBlocks));
    ck(hipMalloc((void **)&ctx->vnorm2, sizeof(double) * (kPmax + 1)));
    ck(hipMalloc((void **)&ctx->ctl, sizeof(PhiCtl)));
    ck(hipHostMalloc((void **)&ctx->dec_host, sizeof(Decision), hipHostMallocDefault));
    ck(hipHostMalloc((void **)&ctx->vn_host, sizeof(double) * (kPmax + 1), hipHostMallocDefault));
    if (rc) {
        free_all(ctx);
        delete ctx;
        return XRB_ENOMEM;
    }
    double *g = (double *)ctx->geo_mem;
    const std::vector<double> *srcs[7] = {&geo.ax, &geo.ay, &geo.az, &geo.bx, &geo.by, &geo.bz, &geo.cl};
    double *dst[7];
    for (int k = 0; k < 7; ++k) {
        dst[k] = g + (size_t)k * 6 * nd;
        ck(hipMemcpy(dst[k], srcs[k]->data(), sizeof(double) * 6 * nd, hipMemcpyHostToDevice));
    }
    double *cellf = g + 7 * 6 * nd;
    const std::vector<double> *cs[4] = {&geo.nx, &geo.ny, &geo.nz, &geo.cor};
    for (int k = 0; k < 4; ++k)
        ck(hipMemcpy(cellf + k * nd, cs[k]->data(), sizeof(double) * nd, hipMemcpyHostToDevice));
    int32_t *nb = (int32_t *)(g + dbl);
    ck(hipMemcpy(nb, geo.nbr.data(), sizeof(int32_t) * 6 * nd, hipMemcpyHostToDevice));
    ck(hipMemset(ctx->ctl, 0, sizeof(PhiCtl)));
    ck(hipMemset(ctx->stage, 0, sizeof(double) * n4 * S_COUNT));
    ck(hipMemset(ctx->V, 0, sizeof(double) * n4 * (params->m_max + 1)));
    if (rc) {
        free_all(ctx);
        delete ctx;
        return XRB_EDEVICE;
    }
    DevMesh &M = ctx->M;
    M.n = n;
    M.nbr = nb;
    M.ax = dst[0]; M.ay = dst[1]; M.az = dst[2];
    M.bx = dst[3]; M.by = dst[4]; M.bz = dst[5];
    M.cl = dst[6];
    M.nx = cellf; M.ny = cellf + nd; M.nz = cellf + 2 * nd; M.cor = cellf + 3 * nd;
    M.nu = geo.nu;
    M.g = params->gravity;
    *out = ctx;
    return XRB_OK;
}

xrb_status xrb_destroy(xrb_ctx *ctx) {
    if (!ctx) return XRB_EINVAL;
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    const int rc = free_all(ctx);
    delete ctx;
    return (e != hipSuccess || rc) ? XRB_EDEVICE : XRB_OK;
}

xrb_status xrb_set_stream(xrb_ctx *ctx, void *stream) {
    if (!ctx) return XRB_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return XRB_OK;
}

xrb_status xrb_sync(xrb_ctx *ctx) {
    if (!ctx) return XRB_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return XRB_OK;
}

const char *xrb_last_error(const xrb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t xrb_n_cells(const xrb_ctx *ctx) { return ctx ? ctx->n : 0; }

xrb_status xrb_rhs(xrb_ctx *ctx, const double *u, double *f) {
    if (!ctx || !u || !f || u == f) return (xrb_status)fail(ctx, XRB_EINVAL, "rhs: bad pointers");
    rhs_plain(ctx, u, f);
    HIPCHK(hipGetLastError());
    return XRB_OK;
}

xrb_status xrb_jv(xrb_ctx *ctx, const double *u, const double *v, double *jv) {
    if (!ctx || !u || !v || !jv || jv == u || jv == v)
        return (xrb_status)fail(ctx, XRB_EINVAL, "jv: bad pointers");
    launch_linearize(ctx->M, u, ctx->eta, ctx->stream);
    jv_plain(ctx, u, v, jv, 1.0);
    HIPCHK(hipGetLastError());
    return XRB_OK;
}

xrb_status xrb_phi_combo(xrb_ctx *ctx, double dt, const double *u, int p, const double *const *v,
                         int ns, const double *rho, double *const *w_out, xrb_phi_stats *stats) {
    if (!ctx || !u) return (xrb_status)fail(ctx, XRB_EINVAL, "phi_combo: null");
    if (!(dt == dt)) return (xrb_status)fail(ctx, XRB_EINVAL, "phi_combo: dt");
    for (int i = 0; i < ns && w_out; ++i)
        if (w_out[i] == u) return (xrb_status)fail(ctx, XRB_EINVAL, "phi_combo: output aliases u");
    launch_linearize(ctx->M, u, ctx->eta, ctx->stream);
    int rc = phi_run(ctx, dt, u, p, v, ns, rho, w_out, 0, nullptr, stats);
    if (rc == XRB_OK) HIPCHK(hipGetLastError());
    return (xrb_status)rc;
}

xrb_status xrb_step(xrb_ctx *ctx, xrb_method method, double *u, double dt) {
    if (!ctx || !u || !(dt > 0.0)) return (xrb_status)fail(ctx, XRB_EINVAL, "step: bad argument");
    const hipStream_t s = ctx->stream;
    double *Fn = ctx->sv(S_FN), *v = ctx->sv(S_V), *W1 = ctx->sv(S_W1), *W2 = ctx->sv(S_W2);
    double *X1 = ctx->sv(S_X1), *X2 = ctx->sv(S_X2), *U2 = ctx->sv(S_U2), *U3 = ctx->sv(S_U3);
    double *D2 = ctx->sv(S_D2), *D3 = ctx->sv(S_D3), *a3 = ctx->sv(S_A3), *a4 = ctx->sv(S_A4);
    double *t1 = ctx->sv(S_T1), *t2 = ctx->sv(S_T2);
    for (auto &st : ctx->last_stats) st = xrb_phi_stats{};
    rhs_plain(ctx, u, Fn);
    lincomb(ctx, v, {Fn}, {dt});
    launch_linearize(ctx->M, u, ctx->eta, s);
    // D = F(U) - Fn - J_n (U - u_n)
    auto nonlin = [&](const double *U, double *D) {
        lincomb(ctx, t1, {U, u}, {1.0, -1.0});
        jv_plain(ctx, u, t1, t2, 1.0);
        rhs_plain(ctx, U, D);
        lincomb(ctx, D, {D, Fn, t2}, {1.0, -1.0, -1.0});
    };
    int rc = XRB_OK;
    if (method == XRB_EXPRB42) {
        const double r1[1] = {0.75}, r2[1] = {1.0};
        const double *vi[2] = {nullptr, v};
        double *o1[1] = {W1};
        rc = phi_run(ctx, dt, u, 1, vi, 1, r1, o1, ctx->m_warm[0], &ctx->m_warm[0], &ctx->last_stats[0]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, U2, {u, W1}, {1.0, 1.0});
        nonlin(U2, D2);
        lincomb(ctx, a3, {D2}, {32.0 / 9.0 * dt});
        const double *vii[4] = {nullptr, v, nullptr, a3};
        double *o2[1] = {W2};
        rc = phi_run(ctx, dt, u, 3, vii, 1, r2, o2, ctx->m_warm[1], &ctx->m_warm[1], &ctx->last_stats[1]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, u, {u, W2}, {1.0, 1.0});
    } else if (method == XRB_PEXPRB43) {
        const double r1[2] = {0.5, 1.0}, r2[1] = {1.0};
        const double *vi[2] = {nullptr, v};
        double *o1[2] = {W1, W2};
        rc = phi_run(ctx, dt, u, 1, vi, 2, r1, o1, ctx->m_warm[0], &ctx->m_warm[0], &ctx->last_stats[0]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, U2, {u, W1}, {1.0, 1.0});
        lincomb(ctx, U3, {u, W2}, {1.0, 1.0});
        nonlin(U2, D2);
        nonlin(U3, D3);
        lincomb(ctx, a3, {D2, D3}, {16.0 * dt, -2.0 * dt});
        lincomb(ctx, a4, {D2, D3}, {-48.0 * dt, 12.0 * dt});
        const double *vii[5] = {nullptr, nullptr, nullptr, a3, a4};
        double *o2[1] = {X1};
        rc = phi_run(ctx, dt, u, 4, vii, 1, r2, o2, ctx->m_warm[1], &ctx->m_warm[1], &ctx->last_stats[1]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, u, {U3, X1}, {1.0, 1.0});
    } else if (method == XRB_EXPRB53) {
        const double r1[2] = {0.5, 0.9}, r3[1] = {1.0};
        const double *vi[2] = {nullptr, v};
        double *o1[2] = {W1, W2};
        rc = phi_run(ctx, dt, u, 1, vi, 2, r1, o1, ctx->m_warm[0], &ctx->m_warm[0], &ctx->last_stats[0]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, U2, {u, W1}, {1.0, 1.0});
        nonlin(U2, D2);
        lincomb(ctx, a3, {D2}, {dt});
        const double *vii[4] = {nullptr, nullptr, nullptr, a3};
        double *o2[2] = {X1, X2};
        rc = phi_run(ctx, dt, u, 3, vii, 2, r1, o2, ctx->m_warm[1], &ctx->m_warm[1], &ctx->last_stats[1]);
        if (rc) return (xrb_status)rc;
        // U3 = u + W(i)_2 + (27/25)(2^3) W(ii)_1 + (729/125)(10/9)^3 W(ii)_2
        lincomb(ctx, U3, {u, W2, X1, X2}, {1.0, 1.0, 216.0 / 25.0, 8.0});
        nonlin(U3, D3);
        lincomb(ctx, a3, {D2, D3}, {18.0 * dt, -250.0 / 81.0 * dt});
        lincomb(ctx, a4, {D2, D3}, {-60.0 * dt, 500.0 / 27.0 * dt});
        const double *viii[5] = {nullptr, v, nullptr, a3, a4};
        double *o3[1] = {W1};
        rc = phi_run(ctx, dt, u, 4, viii, 1, r3, o3, ctx->m_warm[2], &ctx->m_warm[2], &ctx->last_stats[2]);
        if (rc) return (xrb_status)rc;
        lincomb(ctx, u, {u, W1}, {1.0, 1.0});
    } else if (method == XRB_EPI3 || method == XRB_EPI2) {
        const double r1[1] = {1.0};
        double *uprev = ctx->sv(S_UPREV), *fprev = ctx->sv(S_FPREV);
        double *o1[1] = {W1};
        if (method == XRB_EPI3 && ctx->have_prev) {
            // R_{n-1} = F(u_{n-1}) - F(u_n) - J_n (u_{n-1} - u_n)
            lincomb(ctx, t1, {uprev, u}, {1.0, -1.0});
            jv_plain(ctx, u, t1, t2, 1.0);
            lincomb(ctx, a3, {fprev, Fn, t2}, {2.0 / 3.0 * dt, -2.0 / 3.0 * dt, -2.0 / 3.0 * dt});
            const double *vi[3] = {nullptr, v, a3};
            rc = phi_run(ctx, dt, u, 2, vi, 1, r1, o1, ctx->m_warm[0], &ctx->m_warm[0], &ctx->last_stats[0]);
        } else {
            const double *vi[2] = {nullptr, v};
            rc = phi_run(ctx, dt, u, 1, vi, 1, r1, o1, ctx->m_warm[1], &ctx->m_warm[1], &ctx->last_stats[1]);
        }
        if (rc) return (xrb_status)rc;
        HIPCHK(hipMemcpyAsync(uprev, u, sizeof(double) * ctx->n4, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(fprev, Fn, sizeof(double) * ctx->n4, hipMemcpyDeviceToDevice, s));
        ctx->have_prev = 1;
        lincomb(ctx, u, {u, W1}, {1.0, 1.0});
    } else {
        return (xrb_status)fail(ctx, XRB_EINVAL, "step: unknown method");
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    prof_drain(ctx);
    return XRB_OK;
}

xrb_status xrb_step_stats(const xrb_ctx *ctx, xrb_phi_stats *out3) {
    if (!ctx || !out3) return XRB_EINVAL;
    for (int k = 0; k < 3; ++k) out3[k] = ctx->last_stats[k];
    return XRB_OK;
}

xrb_status xrb_reset_history(xrb_ctx *ctx) {
    if (!ctx) return XRB_EINVAL;
    ctx->m_warm[0] = ctx->m_warm[1] = ctx->m_warm[2] = 0;
    ctx->have_prev = 0;
    ctx->sched.clear();
    ctx->sched_pos = 0;
    return XRB_OK;
}

xrb_status xrb_schedule_mode(xrb_ctx *ctx, int mode) {
    if (!ctx || mode < XRB_FREE || mode > XRB_REPLAY) return XRB_EINVAL;
    ctx->mode = mode;
    ctx->sched_pos = 0;
    return XRB_OK;
}

xrb_status xrb_schedule_set(xrb_ctx *ctx, const double *entries, int len) {
    if (!ctx || len < 0 || (len > 0 && !entries)) return XRB_EINVAL;
    ctx->sched.resize(len);
    for (int i = 0; i < len; ++i)
        ctx->sched[i] = {entries[3 * i], (int32_t)entries[3 * i + 1], (int32_t)entries[3 * i + 2]};
    ctx->sched_pos = 0;
    return XRB_OK;
}

xrb_status xrb_schedule_get(const xrb_ctx *ctx, double *entries, int cap, int *len) {
    if (!ctx || !len || cap < 0 || (cap > 0 && !entries)) return XRB_EINVAL;
    const int L = (int)ctx->sched.size();
    *len = L;
    for (int i = 0; i < L && i < cap; ++i) {
        entries[3 * i] = ctx->sched[i].tau;
        entries[3 * i + 1] = ctx->sched[i].m;
        entries[3 * i + 2] = ctx->sched[i].flags;
    }
    return XRB_OK;
}

xrb_status xrb_profile(xrb_ctx *ctx, int enable) {
    if (!ctx) return XRB_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    prof_drain(ctx);
    ctx->prof_every = enable > 0 ? enable : 0;
    if (enable > 0)
        for (int k = 0; k < XRB_K_COUNT; ++k) {
            ctx->prof_ms[k] = 0.0;
            ctx->prof_n[k] = 0;
            ctx->prof_seen[k] = 0;
        }
    return XRB_OK;
}

xrb_status xrb_profile_get(const xrb_ctx *ctx, int kernel, double *timed_ms, int64_t *timed,
                           int64_t *launches) {
    if (!ctx || kernel < 0 || kernel >= XRB_K_COUNT || !timed_ms || !timed || !launches)
        return XRB_EINVAL;
    *timed_ms = ctx->prof_ms[kernel];
    *timed = ctx->prof_n[kernel];
    *launches = ctx->prof_seen[kernel];
    return XRB_OK;
}

}  // extern "C"
