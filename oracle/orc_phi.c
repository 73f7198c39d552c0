/*
 * Oracle: phipm_simul_iom2 (Alg. 1 of Sec. 4.3).  TEST INFRASTRUCTURE ONLY.
 *
 * Computes W_i = sum_{l=0}^p rho_i^l phi_l(rho_i A) v_l for 0 < rho_1 < ... <=
 * 1, i.e. the solution at t = rho_i of y' = A y + sum_{j>=1} t^(j-1)/(j-1)!
 * v_j, y(0) = v_0 (eq. 3.15), by adaptive substeps t_k -> t_k + tau (eq.
 * 3.17 with the w_j recurrence 3.18), each substep needing one Krylov
 * approximation of phi_p(tau A) w_p built by the incomplete orthogonalisation
 * method with orthogonalisation length 2 (IOM2).
 *
 * Steps, in the order of Alg. 1:
 *   1. w_0 = y_k, w_j = A w_{j-1} + sum_{l=0}^{p-j} t_k^l/l! v_{j+l}; the
 *      product A w_{j-1} is skipped when w_{j-1} is known to be zero
 *      (the second modification of Sec. 4.3).
 *   2. beta = ||w_p||, IOM2 basis V_{m+1}, banded H_m, h_{m+1,m};
 *      X = exp(tau Hhat), Hhat = [[H_m, e_1 e_1^T], [0, N_{p+1}]].
 *   3. eps = beta h_{m+1,m} |X(m, m+p+1)| (the correction term's size).
 *   4.-5. (tau, m) update and cost comparison (eq. cost).
 *   6. accept iff omega = t_out eps / (tau Tol) <= delta, then
 *      y_{k+1} = sum_{j<p} tau^j/j! w_j + beta V_m X(1:m, m+p)
 *                + beta h_{m+1,m} X(m, m+p+1) v_{m+1}.
 *   Outputs are stored when t_k reaches each rho_i exactly (first
 *   modification of Sec. 4.3).
 *
 * Points the paper leaves open, and how this file reads them:
 *   - Tol is relative: Tol_abs = tol * max_l ||v_l||_2; all-zero inputs give W = 0.
 *   - beta is ||w_p|| of the current substep (Alg. 1 prints ||v_0||).
 *   - IOM2 uses classical two-term Gram-Schmidt (both coefficients against the
 *     unmodified A v_j); breakdown when h_{j+1,j} <= 1e-14 ||H_j||_1.
 *   - the correction term and eps carry the tau scaling of X = exp(tau Hhat).
 *   - controller: gamma = 0.8; order estimate q (start max(1, m/4)) from two
 *     consecutive attempts at the same point with equal m; error ratio kappa
 *     (start 2, floor 1.1) from two with equal tau; tau_new = tau (gamma/omega)^(1/q)
 *     clamped to [tau/5, 2 tau] and rounded down to 2 significant digits;
 *     m_new = m + ceil(ln(omega/gamma)/ln kappa) clamped to
 *     [max(1, ceil(3m/4)), min(m_max, floor(4m/3) + 1)]; change tau iff
 *     C(tau_new, m) < C(tau, m_new) (eq. cost with n_A = 40 n, nint = round half
 *     away from zero, the log2 term floored at 0); a rejected attempt whose m
 *     would not change changes tau instead.
 *   - substeps are clamped to land exactly on each rho_i; the controller's own
 *     tau carries over to the next output.
 *   - warm start: each call starts from the Krylov size of the previous call's
 *     last accepted attempt at the same call site.
 *   - caps: 10^4 attempts, tau >= 1e-12 rho_Ns.
 * The HIP library implements the same readings in code of its own.
 */
#include "orc.h"
#include "orc_par.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

void orc_phi_default_opts(orc_phi_opts *o)
{
    o->tol = 1e-10;
    o->m_init = 1;
    o->m_max = 40;
    o->delta = 1.4;
    o->gamma = 0.8;
    o->max_attempts = 10000;
    o->mode = ORC_FREE;
    o->sched = NULL;
    o->tape = NULL;
}

void orc_tape_free(orc_phi_tape *t)
{
    if (!t) return;
    for (int k = 0; k < t->len; k++) {
        free(t->s[k].H);
        free(t->s[k].V);
        free(t->s[k].w);
    }
    free(t->s);
    memset(t, 0, sizeof(*t));
}

/* append the accepted substep [t, t + tau] to the tape */
static int tape_push(orc_phi_tape *tp, int n, int p, double t, double tau, double t_out, int out,
                     int m, double beta, double hsub, const double *H, int ldh,
                     const double *V, const double *wv)
{
    if (tp->len == tp->cap) {
        int nc = tp->cap ? 2 * tp->cap : 16;
        orc_substep *ns = realloc(tp->s, sizeof(orc_substep) * nc);
        if (!ns) return ORC_ENOMEM;
        tp->s = ns;
        tp->cap = nc;
    }
    tp->n = n;
    tp->p = p;
    orc_substep *e = &tp->s[tp->len];
    memset(e, 0, sizeof(*e));
    e->t = t; e->tau = tau; e->t_out = t_out; e->out = out;
    e->m = m; e->beta = beta; e->hsub = hsub;
    e->H = calloc(m > 0 ? (size_t)m * m : 1, sizeof(double));
    e->V = calloc((size_t)(m + 1) * n, sizeof(double));
    e->w = calloc(p > 0 ? (size_t)p * n : 1, sizeof(double));
    if (!e->H || !e->V || !e->w) {
        free(e->H); free(e->V); free(e->w);
        return ORC_ENOMEM;
    }
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) e->H[r * m + c] = H[r * ldh + c];
    if (m > 0) memcpy(e->V, V, sizeof(double) * (size_t)(m + 1) * n);
    if (p > 0) memcpy(e->w, wv, sizeof(double) * (size_t)p * n);
    tp->len++;
    return ORC_OK;
}

static double nrm2(int n, const double *x)
{
    double acc = 0.0;
    for (int i = 0; i < n; i++) acc += x[i] * x[i];
    return sqrt(acc);
}

static double dotp(int n, const double *x, const double *y)
{
    double acc = 0.0;
    for (int i = 0; i < n; i++) acc += x[i] * y[i];
    return acc;
}

/* round x > 0 down to two significant decimal digits, using only exact
 * scalings by 10 so that the result does not depend on a libm */
static double quantise2(double x)
{
    double p = 1.0;
    while (p > x) p /= 10.0;
    while (p * 10.0 <= x) p *= 10.0;
    double unit = p / 10.0;
    return floor(x / unit) * unit;
}

/* eq. cost: the estimated work C(tau, m) of reaching the output time with
 * substeps tau and Krylov size m, remaining = t_out - t, hnorm = ||tau Hhat||_1:
 *   max(1, nint(remaining / tau)) m (n + n_A) + 2 (p - 1)(n_A + n)
 *     + M (m + p + 1)^3 + (2p + 1) n,
 *   M = 44/3 + 2 max(0, nint(log2(hnorm / 5.37))),  n_A = 40 n,
 * nint rounding half away from zero (C's round). */
double orc_phi_cost(double tau, int m, int p, double remaining, double n, double hnorm)
{
    double nA = 40.0 * n;
    double ks = round(remaining / tau);
    if (ks < 1.0) ks = 1.0;
    double M = 44.0 / 3.0;
    if (hnorm > 0.0) {
        double r = round(log2(hnorm / 5.37));
        if (r > 0.0) M += 2.0 * r;
    }
    double K = (double)(m + p + 1);
    return ks * m * (n + nA) + 2.0 * (p - 1) * (nA + n) + M * K * K * K + (2.0 * p + 1.0) * n;
}

static int sched_push(orc_schedule *s, double tau, int m, int flags)
{
    if (s->len == s->cap) {
        int nc = s->cap ? 2 * s->cap : 64;
        orc_attempt *na = realloc(s->a, sizeof(orc_attempt) * nc);
        if (!na) return ORC_ENOMEM;
        s->a = na;
        s->cap = nc;
    }
    s->a[s->len].tau = tau;
    s->a[s->len].m = m;
    s->a[s->len].flags = flags;
    s->len++;
    return ORC_OK;
}

int orc_phi_combo(int n, orc_matvec_fn A, void *actx, int p, const double *const *v,
                  int ns, const double *rho, double *const *w_out,
                  const orc_phi_opts *o, int *m_warm, orc_phi_stats *st)
{
    orc_phi_stats lst;
    if (!st) st = &lst;
    memset(st, 0, sizeof(*st));
    if (n <= 0 || p < 0 || ns < 1 || !rho || !w_out) return ORC_EINVAL;
    for (int i = 0; i < ns; i++)
        if (!(rho[i] > 0.0) || rho[i] > 1.0 || (i > 0 && !(rho[i] > rho[i - 1]))) return ORC_EINVAL;
    int mmax = o->m_max;
    if (mmax < 1) return ORC_EINVAL;

    /* Tol_abs = tol * max_l ||v_l|| ; a zero input gives W = 0 exactly */
    double scale = 0.0;
    for (int l = 0; l <= p; l++)
        if (v[l]) {
            double s = nrm2(n, v[l]);
            if (s != s) return ORC_ENAN;
            if (s > scale) scale = s;
        }
    if (scale == 0.0) {
        for (int i = 0; i < ns; i++) memset(w_out[i], 0, sizeof(double) * n);
        return ORC_OK;
    }
    double tol = o->tol * scale;

    int rc = ORC_OK;
    double *y = calloc(n, sizeof(double));
    double *wv = calloc((size_t)(p + 1) * n, sizeof(double));       /* w_0..w_p */
    double *V = calloc((size_t)(mmax + 1) * n, sizeof(double));     /* basis */
    double *H = calloc((size_t)(mmax + 1) * mmax, sizeof(double));  /* (mmax+1) x mmax */
    int Kmax = mmax + p + 1;
    double *Hh = malloc(sizeof(double) * Kmax * Kmax);
    double *X = malloc(sizeof(double) * Kmax * Kmax);
    int *wzero = calloc(p + 1, sizeof(int));
    if (!y || !wv || !V || !H || !Hh || !X || !wzero) { rc = ORC_ENOMEM; goto done; }

    int y_zero = 1;
    if (v[0]) { memcpy(y, v[0], sizeof(double) * n); y_zero = 0; }
    double t = 0.0;
    double tau = rho[0];
    int m = (m_warm && *m_warm > 0) ? *m_warm : o->m_init;
    if (m < 1) m = 1;
    if (m > mmax) m = mmax;
    double q = m / 4.0 > 1.0 ? m / 4.0 : 1.0;   /* order estimate */
    double kappa = 2.0;                          /* per-dimension error ratio */
    int have_prev = 0, prev_m = 0;
    double prev_tau = 0.0, prev_omega = 0.0;

    int point_ready = 0;   /* w_j / basis built for the current (t, y) */
    int built = 0;         /* number of IOM2 columns built */
    int m_break = 0;       /* happy breakdown: basis size, 0 = none */
    double beta = 0.0;

    for (int io = 0; io < ns; io++) {
        double t_out = rho[io];
        while (t < t_out) {
            if (st->attempts >= o->max_attempts) { rc = ORC_ENOTCONV; goto done; }
            st->attempts++;
            double rem = t_out - t;
            double tau_u;
            int lands;
            if (o->mode == ORC_REPLAY) {
                orc_schedule *s = o->sched;
                if (!s || s->pos >= s->len) { rc = ORC_ESCHED; goto done; }
                tau_u = s->a[s->pos].tau;
                m = s->a[s->pos].m;
                lands = (s->a[s->pos].flags >> 1) & 1;
                if (m < 1 || m > mmax) { rc = ORC_ESCHED; goto done; }
            } else if (tau >= rem * (1.0 - 1e-12)) {
                tau_u = rem;
                lands = 1;
            } else {
                tau_u = tau;
                lands = 0;
            }
            if (!(tau_u >= 1e-12 * rho[ns - 1])) { rc = ORC_ENOTCONV; goto done; }
            const int m_att = m;   /* Krylov size of this attempt */

            /* step 1: w_j recurrence (eq. 3.18) with the zero-skip */
            if (!point_ready) {
                memcpy(wv, y, sizeof(double) * n);
                wzero[0] = y_zero;
                for (int j = 1; j <= p; j++) {
                    double *wj = wv + (size_t)j * n;
                    int z = 1;
                    if (!wzero[j - 1]) {
                        A(actx, wv + (size_t)(j - 1) * n, wj);
                        st->matvecs++;
                        st->rec_matvecs++;
                        z = 0;
                    } else {
                        memset(wj, 0, sizeof(double) * n);
                    }
                    double fac = 1.0;   /* t^l / l! */
                    for (int l = 0; l <= p - j; l++) {
                        if (l > 0) fac = fac * t / l;
                        if (!v[j + l] || (l > 0 && t == 0.0)) continue;
                        ORC_PARFOR
                        for (int k = 0; k < n; k++) wj[k] += fac * v[j + l][k];
                        z = 0;
                    }
                    wzero[j] = z;
                }
                beta = wzero[p] ? 0.0 : nrm2(n, wv + (size_t)p * n);
                if (beta != beta) { rc = ORC_ENAN; goto done; }
                built = 0;
                m_break = 0;
                if (beta > 0.0) {
                    const double *wp = wv + (size_t)p * n;
                    ORC_PARFOR
                    for (int k = 0; k < n; k++) V[k] = wp[k] / beta;
                }
                point_ready = 1;
            }

            int accept;
            double omega = 0.0, eps = 0.0, normH = 0.0;
            int meff = m;
            if (beta == 0.0) {
                /* w_p = 0: the substep is exact, y_{k+1} = sum_{j<p} tau^j/j! w_j */
                accept = 1;
            } else {
                /* step 2(i): IOM2, extended to m columns if needed */
                while (built < m && !m_break) {
                    int j = built;
                    double *w = V + (size_t)(j + 1) * n;
                    A(actx, V + (size_t)j * n, w);
                    st->matvecs++;
                    /* classical two-term Gram-Schmidt: both coefficients
                     * against the unmodified A v_j */
                    double hjj = dotp(n, w, V + (size_t)j * n);
                    double hmj = j > 0 ? dotp(n, w, V + (size_t)(j - 1) * n) : 0.0;
                    ORC_PARFOR
                    for (int k = 0; k < n; k++) w[k] -= hjj * V[(size_t)j * n + k];
                    if (j > 0) {
                        ORC_PARFOR
                        for (int k = 0; k < n; k++) w[k] -= hmj * V[(size_t)(j - 1) * n + k];
                    }
                    H[j * mmax + j] = hjj;
                    if (j > 0) H[(j - 1) * mmax + j] = hmj;
                    double hn = nrm2(n, w);
                    if (hn != hn) { rc = ORC_ENAN; goto done; }
                    /* breakdown test against the 1-norm of the square block */
                    double bn = 0.0;
                    for (int c = 0; c <= j; c++) {
                        double cs = 0.0;
                        for (int r = 0; r <= j; r++) cs += fabs(H[r * mmax + c]);
                        if (cs > bn) bn = cs;
                    }
                    if (hn <= 1e-14 * bn) {
                        H[(j + 1) * mmax + j] = 0.0;
                        memset(w, 0, sizeof(double) * n);
                        m_break = j + 1;
                    } else {
                        H[(j + 1) * mmax + j] = hn;
                        ORC_PARFOR
                        for (int k = 0; k < n; k++) w[k] /= hn;
                    }
                    built++;
                }
                meff = (m_break && m_break < m) ? m_break : m;
                double hsub = (m_break && meff == m_break) ? 0.0 : H[meff * mmax + meff - 1];

                /* step 2(ii): augmented matrix and its exponential */
                int K = meff + p + 1;
                memset(Hh, 0, sizeof(double) * K * K);
                for (int r = 0; r < meff; r++)
                    for (int c = 0; c < meff; c++) Hh[r * K + c] = tau_u * H[r * mmax + c];
                Hh[0 * K + meff] = tau_u;
                for (int k = 0; k < p; k++) Hh[(meff + k) * K + meff + k + 1] = tau_u;
                for (int c = 0; c < K; c++) {
                    double cs = 0.0;
                    for (int r = 0; r < K; r++) cs += fabs(Hh[r * K + c]);
                    if (cs > normH) normH = cs;
                }
                orc_expm(K, Hh, X);
                st->expms++;

                /* step 3: error estimate and acceptance ratio */
                eps = beta * hsub * fabs(X[(meff - 1) * K + meff + p]);
                omega = t_out * eps / (tau_u * tol);
                if (omega != omega) { rc = ORC_ENAN; goto done; }
                if (o->mode == ORC_REPLAY)
                    accept = o->sched->a[o->sched->pos].flags & 1;
                else
                    accept = omega <= o->delta;
            }
            st->sum_m += m_att;
            if (m_att > st->max_m) st->max_m = m_att;

            if (o->mode == ORC_REPLAY) {
                o->sched->pos++;
            } else {
                if (o->mode == ORC_RECORD) {
                    int r2 = sched_push(o->sched, tau_u, m, (accept ? 1 : 0) | (lands ? 2 : 0));
                    if (r2) { rc = r2; goto done; }
                }
                /* steps 4-5: new (tau, m) and the cost comparison */
                if (beta > 0.0) {
                    if (have_prev && omega > 0.0 && prev_omega > 0.0) {
                        if (m_att == prev_m && tau_u != prev_tau) {
                            double qq = log(omega / prev_omega) / log(tau_u / prev_tau);
                            q = qq > 1.0 ? qq : 1.0;
                        } else if (tau_u == prev_tau && m_att != prev_m) {
                            double kk = pow(omega / prev_omega, 1.0 / (prev_m - m_att));
                            kappa = kk > 1.1 ? kk : 1.1;
                        }
                    }
                    double tau_new, mnew_d;
                    if (omega > 0.0) {
                        tau_new = tau_u * pow(o->gamma / omega, 1.0 / q);
                        mnew_d = m_att + ceil(log(omega / o->gamma) / log(kappa));
                    } else {
                        tau_new = 2.0 * tau_u;
                        mnew_d = -1e300;
                    }
                    if (tau_new > 2.0 * tau_u) tau_new = 2.0 * tau_u;
                    if (tau_new < tau_u / 5.0) tau_new = tau_u / 5.0;
                    tau_new = quantise2(tau_new);
                    int lo = (3 * m_att + 3) / 4;
                    if (lo < 1) lo = 1;
                    int hi = (4 * m_att) / 3 + 1;
                    if (hi > mmax) hi = mmax;
                    if (mnew_d < lo) mnew_d = lo;
                    if (mnew_d > hi) mnew_d = hi;
                    int m_new = (int)mnew_d;
                    /* ||tau Hhat||_1 scales linearly with tau */
                    double c_tau = orc_phi_cost(tau_new, m_att, p, t_out - t, (double)n,
                                                normH * tau_new / tau_u);
                    double c_m = orc_phi_cost(tau_u, m_new, p, t_out - t, (double)n,
                                              normH * tau_u / tau_u);
                    int change_tau = c_tau < c_m;
                    /* a rejected attempt must change something */
                    if (!accept && !change_tau && m_new == m_att) change_tau = 1;
                    if (change_tau) tau = tau_new;
                    else m = m_new;
                }
            }

            if (accept) {
                /* y_{k+1} = sum_{j<p} tau^j/j! w_j + Krylov approximation of
                 * tau^p phi_p(tau A) w_p (eq. 3.17, upper limit p-1) */
                double *yn = malloc(sizeof(double) * n);
                if (!yn) { rc = ORC_ENOMEM; goto done; }
                memset(yn, 0, sizeof(double) * n);
                double fac = 1.0;
                for (int j = 0; j < p; j++) {
                    if (j > 0) fac = fac * tau_u / j;
                    if (wzero[j]) continue;
                    const double *wj = wv + (size_t)j * n;
                    ORC_PARFOR
                    for (int k = 0; k < n; k++) yn[k] += fac * wj[k];
                }
                if (beta > 0.0) {
                    int K = meff + p + 1;
                    int cmain = p > 0 ? meff + p - 1 : 0;
                    for (int c = 0; c < meff; c++) {
                        double a = beta * X[c * K + cmain];
                        const double *vc = V + (size_t)c * n;
                        ORC_PARFOR
                        for (int k = 0; k < n; k++) yn[k] += a * vc[k];
                    }
                    double hsub = (m_break && meff == m_break) ? 0.0 : H[meff * mmax + meff - 1];
                    double a = beta * hsub * X[(meff - 1) * K + meff + p];
                    if (a != 0.0) {
                        const double *vc = V + (size_t)meff * n;
                        ORC_PARFOR
                        for (int k = 0; k < n; k++) yn[k] += a * vc[k];
                    }
                }
                memcpy(y, yn, sizeof(double) * n);
                free(yn);
                if (o->tape) {
                    int mt = beta > 0.0 ? meff : 0;
                    double hs = 0.0;
                    if (mt > 0) hs = (m_break && meff == m_break) ? 0.0 : H[meff * mmax + meff - 1];
                    int r3 = tape_push(o->tape, n, p, t, tau_u, t_out, lands ? io : -1, mt, beta,
                                       hs, H, mmax, V, wv);
                    if (r3) { rc = r3; goto done; }
                }
                y_zero = 0;
                t = lands ? t_out : t + tau_u;
                point_ready = 0;
                have_prev = 0;
                st->accepted++;
                st->last_m = m_att;
                if (m_warm) *m_warm = m_att;
            } else {
                st->rejected++;
                have_prev = 1;
                prev_omega = omega;
                prev_tau = tau_u;
                prev_m = m_att;
            }
            (void)eps;
        }
        memcpy(w_out[io], y, sizeof(double) * n);
    }
done:
    free(y); free(wv); free(V); free(H); free(Hh); free(X); free(wzero);
    return rc;
}

/* ------------------------------------------------------------------ */
typedef struct { int n; const double *A; } dense_ctx;

static void dense_mv(void *ctx, const double *x, double *y)
{
    const dense_ctx *d = ctx;
    for (int i = 0; i < d->n; i++) {
        double acc = 0.0;
        for (int j = 0; j < d->n; j++) acc += d->A[(size_t)i * d->n + j] * x[j];
        y[i] = acc;
    }
}

int orc_phi_combo_dense(int n, const double *A, int p, const double *const *v, int ns,
                        const double *rho, double *const *w_out, const orc_phi_opts *o,
                        int *m_warm, orc_phi_stats *st)
{
    dense_ctx d = {n, A};
    return orc_phi_combo(n, dense_mv, &d, p, v, ns, rho, w_out, o, m_warm, st);
}
