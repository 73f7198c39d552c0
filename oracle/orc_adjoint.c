/*
 * Oracle: adjoints of the phi-combination and of an exprb42 step.
 * TEST INFRASTRUCTURE ONLY.
 *
 * The paper has no adjoint; this is the continuous adjoint of the ODE that
 * defines the phi-combination (eq. 3.15), evaluated on the substeps of the
 * forward solve.  For
 *   y' = A y + g(t),  g(t) = sum_{j>=1} t^(j-1)/(j-1)! v_j,  y(0) = v_0,
 *   W_i = y(rho_i)
 * and cotangents Wbar_i, the adjoint state mu solves mu' = -A^T mu backwards
 * from mu(rho_ns) = Wbar_ns, jumping by Wbar_i at each earlier rho_i.  Then
 *   vbar_0 = mu(0),   vbar_j = int_0^rho_ns mu(t) t^(j-1)/(j-1)! dt,
 *   <Abar, E> = int_0^rho_ns mu(t)^T E y(t) dt.
 * For A = dt J(u) the last term gives dt int K(mu(t), y(t)) dt with
 * K(a, b) = grad_u <a, J(u) b>.
 *
 * Per forward substep [t_k, t_k + tau] (taken from the tape, in reverse):
 *   - mu_{k+1} = beta_mu v_1 starts an IOM2 Krylov space of A^T (classical
 *     two-term Gram-Schmidt, same breakdown test as the forward);
 *   - X = exp(tau G), G = [[Hbar, e_1 e_1^T], [0, N_p]] with the corrected
 *     Hbar = [[H_m, 0], [h_{m+1,m} e_m^T, 0]] gives
 *       mu_k = beta_mu V_{m+1} X(:, 1)                (= e^{tau A^T} mu_{k+1})
 *       I_l  = beta_mu V_{m+1} X(:, m+2+l)            (= tau^(l+1) phi_{l+1}(tau A^T) mu_{k+1}
 *                                                        = int_0^tau mu(t_k+s) s^l/l! ds)
 *     and vbar_j += sum_{l<j} t_k^(j-1-l)/(j-1-l)! I_l;
 *   - Krylov size: start from the forward's m of the substep; while
 *     omega = t_out beta_mu |X(m+1, 1)| / (tau Tol) > delta, grow m to
 *     max(m+1, floor(4m/3)+1) up to m_max (the tau grid is the forward's);
 *   - the A-term: mu(t_k+s) = beta_mu V^mu a(tau-s), a(r) = exp(r Hbar^mu) e_1,
 *     y(t_k+s) = What b(s), b(s) = exp(s Hhat') e_last, What = [beta V^y_{m+1},
 *     w_{p-1}, .., w_0] (see orc_substep).  M = int_0^tau a(tau-s) b(s)^T ds is
 *     the top-right block of exp(tau [[Hbar^mu, e_1 e_last^T], [0, Hhat'^T]])
 *     (Van Loan), and int K(mu, y) = beta_mu sum_r K(v^mu_r, Z_r), Z = What M^T.
 * Tolerance: Tol = tol * max_i ||Wbar_i||.  A call whose forward inputs were
 * all zero has no substeps; its adjoint then takes one substep per output
 * interval.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

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

/* IOM2 basis of a matvec, grown column by column (same steps as the forward) */
typedef struct {
    int n, mmax, built, brk;
    double *V;   /* (mmax+1) x n */
    double *H;   /* (mmax+1) x mmax */
} krylov;

static int krylov_grow(krylov *K, orc_matvec_fn A, void *actx, int m, orc_phi_stats *st)
{
    int n = K->n, mmax = K->mmax;
    while (K->built < m && !K->brk) {
        int j = K->built;
        double *w = K->V + (size_t)(j + 1) * n;
        A(actx, K->V + (size_t)j * n, w);
        st->matvecs++;
        double hjj = dotp(n, w, K->V + (size_t)j * n);
        double hmj = j > 0 ? dotp(n, w, K->V + (size_t)(j - 1) * n) : 0.0;
        for (int k = 0; k < n; k++) w[k] -= hjj * K->V[(size_t)j * n + k];
        if (j > 0)
            for (int k = 0; k < n; k++) w[k] -= hmj * K->V[(size_t)(j - 1) * n + k];
        K->H[j * mmax + j] = hjj;
        if (j > 0) K->H[(j - 1) * mmax + j] = hmj;
        double hn = nrm2(n, w);
        if (hn != hn) return ORC_ENAN;
        double bn = 0.0;
        for (int c = 0; c <= j; c++) {
            double cs = 0.0;
            for (int r = 0; r <= j; r++) cs += fabs(K->H[r * mmax + c]);
            if (cs > bn) bn = cs;
        }
        if (hn <= 1e-14 * bn) {
            K->H[(j + 1) * mmax + j] = 0.0;
            memset(w, 0, sizeof(double) * n);
            K->brk = j + 1;
        } else {
            K->H[(j + 1) * mmax + j] = hn;
            for (int k = 0; k < n; k++) w[k] /= hn;
        }
        K->built++;
    }
    return ORC_OK;
}

int orc_phi_adjoint(int n, orc_matvec_fn AT, void *atctx, orc_kacc_fn Kf, void *kctx,
                    double *kacc, const orc_phi_tape *tape, int p, int ns, const double *rho,
                    const double *const *wbar, double *const *vbar, const orc_phi_opts *o,
                    orc_phi_stats *st)
{
    orc_phi_stats lst;
    if (!st) st = &lst;
    memset(st, 0, sizeof(*st));
    if (n <= 0 || p < 1 || p > 8 || ns < 1 || !rho || !wbar || !tape) return ORC_EINVAL;
    for (int i = 0; i < ns; i++)
        if (!(rho[i] > 0.0) || rho[i] > 1.0 || (i > 0 && !(rho[i] > rho[i - 1]))) return ORC_EINVAL;
    if (tape->len > 0 && (tape->p != p || tape->n != n)) return ORC_EINVAL;
    int mmax = o->m_max;
    if (mmax < 1) return ORC_EINVAL;
    for (int l = 0; l <= p; l++)
        if (vbar && vbar[l]) memset(vbar[l], 0, sizeof(double) * n);

    double scale = 0.0;
    for (int i = 0; i < ns; i++) {
        double s = nrm2(n, wbar[i]);
        if (s != s) return ORC_ENAN;
        if (s > scale) scale = s;
    }
    if (scale == 0.0) return ORC_OK;
    double tol = o->tol * scale;

    /* the substeps: the forward's, or one per output interval */
    int nsub = tape->len;
    orc_substep *subs = tape->s;
    orc_substep *own = NULL;
    if (nsub == 0) {
        own = calloc(ns, sizeof(orc_substep));
        if (!own) return ORC_ENOMEM;
        for (int i = 0; i < ns; i++) {
            own[i].t = i ? rho[i - 1] : 0.0;
            own[i].tau = rho[i] - own[i].t;
            own[i].t_out = rho[i];
            own[i].out = i;
            own[i].m = 0;
        }
        nsub = ns;
        subs = own;
    }

    int rc = ORC_OK;
    int Gmax = mmax + 1 + p, Tmax = (mmax + 1) + (mmax + 1 + p);
    krylov K = {n, mmax, 0, 0, NULL, NULL};
    K.V = calloc((size_t)(mmax + 1) * n, sizeof(double));
    K.H = calloc((size_t)(mmax + 1) * mmax, sizeof(double));
    double *mu = calloc(n, sizeof(double));
    double *mk = calloc(n, sizeof(double));
    double *I = calloc((size_t)p * n, sizeof(double));
    double *Z = calloc(n, sizeof(double));
    double *G = malloc(sizeof(double) * Gmax * Gmax);
    double *X = malloc(sizeof(double) * Gmax * Gmax);
    double *T = malloc(sizeof(double) * Tmax * Tmax);
    double *E = malloc(sizeof(double) * Tmax * Tmax);
    if (!K.V || !K.H || !mu || !mk || !I || !Z || !G || !X || !T || !E) { rc = ORC_ENOMEM; goto done; }

    for (int k = nsub - 1; k >= 0; k--) {
        const orc_substep *sb = &subs[k];
        if (sb->out >= 0)
            for (int i = 0; i < n; i++) mu[i] += wbar[sb->out][i];
        double bmu = nrm2(n, mu);
        if (bmu != bmu) { rc = ORC_ENAN; goto done; }
        if (bmu == 0.0) continue;
        double tau = sb->tau;

        /* Krylov space of A^T from mu_{k+1} */
        K.built = 0;
        K.brk = 0;
        memset(K.H, 0, sizeof(double) * (mmax + 1) * mmax);
        for (int i = 0; i < n; i++) K.V[i] = mu[i] / bmu;
        int m = sb->m > 0 ? sb->m : o->m_init;
        if (m < 1) m = 1;
        if (m > mmax) m = mmax;
        int me, a;
        for (;;) {
            rc = krylov_grow(&K, AT, atctx, m, st);
            if (rc) goto done;
            me = (K.brk && K.brk < m) ? K.brk : m;
            double h = (K.brk && me == K.brk) ? 0.0 : K.H[me * mmax + me - 1];
            a = me + 1;
            int g = a + p;
            memset(G, 0, sizeof(double) * g * g);
            for (int r = 0; r < me; r++)
                for (int c = 0; c < me; c++) G[r * g + c] = tau * K.H[r * mmax + c];
            G[me * g + me - 1] = tau * h;
            G[0 * g + a] = tau;
            for (int l = 0; l + 1 < p; l++) G[(a + l) * g + a + l + 1] = tau;
            orc_expm(g, G, X);
            st->expms++;
            st->attempts++;
            double eps = bmu * fabs(X[me * g + 0]);
            double omega = sb->t_out * eps / (tau * tol);
            if (omega != omega) { rc = ORC_ENAN; goto done; }
            if (omega <= o->delta || K.brk || m == mmax) {
                if (omega > o->delta && !K.brk) st->rejected++;   /* accepted at m_max */
                break;
            }
            int mn = (4 * m) / 3 + 1;
            if (mn < m + 1) mn = m + 1;
            m = mn > mmax ? mmax : mn;
        }
        st->accepted++;
        st->sum_m += me;
        if (me > st->max_m) st->max_m = me;
        st->last_m = me;
        int g = a + p;

        /* mu_k and the moment integrals I_l */
        memset(mk, 0, sizeof(double) * n);
        memset(I, 0, sizeof(double) * (size_t)p * n);
        for (int r = 0; r < a; r++) {
            const double *vr = K.V + (size_t)r * n;
            double c0 = bmu * X[r * g + 0];
            for (int i = 0; i < n; i++) mk[i] += c0 * vr[i];
            for (int l = 0; l < p; l++) {
                double cl = bmu * X[r * g + a + l];
                double *Il = I + (size_t)l * n;
                for (int i = 0; i < n; i++) Il[i] += cl * vr[i];
            }
        }
        for (int j = 1; j <= p; j++) {
            if (!vbar || !vbar[j]) continue;
            for (int l = 0; l < j; l++) {
                /* t_k^(j-1-l) / (j-1-l)! */
                double f = 1.0;
                for (int q = 1; q <= j - 1 - l; q++) f = f * sb->t / q;
                if (f == 0.0) continue;
                const double *Il = I + (size_t)l * n;
                for (int i = 0; i < n; i++) vbar[j][i] += f * Il[i];
            }
        }

        /* the A-term on this substep */
        if (Kf && kacc && tape->len > 0) {
            int my = sb->m;
            int b = my + 1 + p;
            int tt = a + b;
            memset(T, 0, sizeof(double) * tt * tt);
            for (int r = 0; r < me; r++)
                for (int c = 0; c < me; c++) T[r * tt + c] = tau * K.H[r * mmax + c];
            {
                double h = (K.brk && me == K.brk) ? 0.0 : K.H[me * mmax + me - 1];
                T[me * tt + me - 1] = tau * h;
            }
            /* Hhat' of the forward substep, transposed, in the lower-right block */
            double Hy[64 * 64];
            int bb = b;
            if (bb > 64) { rc = ORC_EINVAL; goto done; }
            memset(Hy, 0, sizeof(double) * bb * bb);
            for (int r = 0; r < my; r++)
                for (int c = 0; c < my; c++) Hy[r * bb + c] = sb->H[r * my + c];
            if (my > 0) Hy[my * bb + my - 1] = sb->hsub;
            Hy[0 * bb + my + 1] = 1.0;
            for (int l = 0; l + 1 < p; l++) Hy[(my + 1 + l) * bb + my + 2 + l] = 1.0;
            for (int r = 0; r < b; r++)
                for (int c = 0; c < b; c++) T[(a + r) * tt + a + c] = tau * Hy[c * bb + r];
            T[0 * tt + a + b - 1] = tau;
            orc_expm(tt, T, E);
            st->expms++;
            for (int r = 0; r < a; r++) {
                memset(Z, 0, sizeof(double) * n);
                int any = 0;
                for (int c = 0; c < b; c++) {
                    double mrc = E[r * tt + a + c];
                    if (mrc == 0.0) continue;
                    const double *wc;
                    double f;
                    if (c <= my) {
                        wc = sb->V + (size_t)c * n;
                        f = sb->beta * mrc;
                    } else {
                        wc = sb->w + (size_t)(p - (c - my)) * n;
                        f = mrc;
                    }
                    if (f == 0.0) continue;
                    for (int i = 0; i < n; i++) Z[i] += f * wc[i];
                    any = 1;
                }
                if (any) Kf(kctx, K.V + (size_t)r * n, Z, bmu, kacc);
            }
        }
        memcpy(mu, mk, sizeof(double) * n);
    }
    if (vbar && vbar[0]) memcpy(vbar[0], mu, sizeof(double) * n);
done:
    free(own);
    free(K.V); free(K.H); free(mu); free(mk); free(I); free(Z); free(G); free(X); free(T); free(E);
    return rc;
}

/* ------------------------------------------------------------------ */
/* dense-matrix form: forward with tape, then the adjoint with           */
/* Abar += scale a b^T                                                   */
/* ------------------------------------------------------------------ */
typedef struct { int n; const double *A; int trans; } dmat;

static void dmv(void *ctx, const double *x, double *y)
{
    const dmat *d = ctx;
    int n = d->n;
    for (int i = 0; i < n; i++) {
        double acc = 0.0;
        if (d->trans)
            for (int j = 0; j < n; j++) acc += d->A[(size_t)j * n + i] * x[j];
        else
            for (int j = 0; j < n; j++) acc += d->A[(size_t)i * n + j] * x[j];
        y[i] = acc;
    }
}

static void outer_acc(void *ctx, const double *a, const double *b, double scale, double *acc)
{
    int n = *(const int *)ctx;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) acc[(size_t)i * n + j] += scale * a[i] * b[j];
}

int orc_phi_vjp_dense(int n, const double *A, int p, const double *const *v, int ns,
                      const double *rho, const double *const *wbar, double *const *w_out,
                      double *const *vbar, double *Abar, const orc_phi_opts *o,
                      orc_phi_stats *fwd, orc_phi_stats *adj)
{
    orc_phi_tape tape;
    memset(&tape, 0, sizeof(tape));
    orc_phi_opts of = *o;
    of.tape = &tape;
    dmat d = {n, A, 0};
    int mw = 0;
    int rc = orc_phi_combo(n, dmv, &d, p, v, ns, rho, w_out, &of, &mw, fwd);
    if (rc) { orc_tape_free(&tape); return rc; }
    dmat dt = {n, A, 1};
    int nn = n;
    if (Abar) memset(Abar, 0, sizeof(double) * (size_t)n * n);
    rc = orc_phi_adjoint(n, dmv, &dt, Abar ? outer_acc : NULL, &nn, Abar, &tape, p, ns, rho,
                         wbar, vbar, o, adj);
    orc_tape_free(&tape);
    return rc;
}

/* ------------------------------------------------------------------ */
/* exprb42 step: u_{n+1} = u_n + W2, with (A = dt J_n, v = dt F_n)        */
/*   W1 = 3/4 phi_1(3/4 A) v,  U2 = u_n + W1,  e = U2 - u_n,              */
/*   D2 = F(U2) - F_n - J_n e,  W2 = phi_1(A) v + phi_3(A) 32/9 dt D2.    */
/* Reverse, with every intermediate its own variable:                     */
/*   call 2: vbar2 = adjoint(Wbar = ubar_{n+1}); ubar_n = ubar_{n+1}      */
/*   Dbar = 32/9 dt vbar2_3;  Ubar2 = (J(U2) - J_n)^T Dbar;               */
/*   Fbar = dt vbar2_1 - Dbar;  ubar_n += J_n^T Dbar - K(Dbar, e)         */
/*   call 1: vbar1 = adjoint(Wbar = Ubar2);  ubar_n += Ubar2;             */
/*   Fbar += dt vbar1_1;  ubar_n += J_n^T Fbar + dt (A-terms of both calls) */
/* ------------------------------------------------------------------ */
typedef struct { const orc_swe *m; const double *u; double dt; int trans; } swe_mv;

static void swe_mv_fn(void *ctx, const double *x, double *y)
{
    const swe_mv *c = ctx;
    if (c->trans) orc_jtv(c->m, c->u, x, y);
    else orc_jv(c->m, c->u, x, y);
    int N = 4 * c->m->n;
    for (int i = 0; i < N; i++) y[i] *= c->dt;
}

typedef struct { const orc_swe *m; double dt; double *tmp; } swe_k;

static void swe_k_fn(void *ctx, const double *a, const double *b, double scale, double *acc)
{
    const swe_k *c = ctx;
    orc_ktv(c->m, a, b, c->tmp);
    int N = 4 * c->m->n;
    double f = scale * c->dt;
    for (int i = 0; i < N; i++) acc[i] += f * c->tmp[i];
}

int orc_step_vjp(const orc_swe *m, int method, const double *u, double dt,
                 const double *ubar_np1, double *ubar_n, const orc_phi_opts *o,
                 orc_phi_stats *adj)
{
    if (method != ORC_EXPRB42) return ORC_EINVAL;
    int N = 4 * m->n;
    int rc = ORC_OK;
    orc_phi_stats lst[2];
    if (!adj) adj = lst;
    orc_phi_tape t1, t2;
    memset(&t1, 0, sizeof(t1));
    memset(&t2, 0, sizeof(t2));
    double *Fn = calloc(N, sizeof(double)), *v = calloc(N, sizeof(double));
    double *W1 = calloc(N, sizeof(double)), *W2 = calloc(N, sizeof(double));
    double *U2 = calloc(N, sizeof(double)), *e = calloc(N, sizeof(double));
    double *D2 = calloc(N, sizeof(double)), *a3 = calloc(N, sizeof(double));
    double *t = calloc(N, sizeof(double)), *Dbar = calloc(N, sizeof(double));
    double *Ubar2 = calloc(N, sizeof(double)), *Fbar = calloc(N, sizeof(double));
    double *kacc = calloc(N, sizeof(double)), *ktmp = calloc(N, sizeof(double));
    double *vb[4] = {NULL, calloc(N, sizeof(double)), NULL, calloc(N, sizeof(double))};
    if (!Fn || !v || !W1 || !W2 || !U2 || !e || !D2 || !a3 || !t || !Dbar || !Ubar2 || !Fbar ||
        !kacc || !ktmp || !vb[1] || !vb[3]) { rc = ORC_ENOMEM; goto out; }

    /* forward, recording both calls */
    swe_mv A = {m, u, dt, 0}, AT = {m, u, dt, 1};
    swe_k kc = {m, dt, ktmp};
    orc_rhs(m, u, Fn);
    for (int i = 0; i < N; i++) v[i] = dt * Fn[i];
    {
        orc_phi_opts o1 = *o;
        o1.tape = &t1;
        double rho1[1] = {0.75};
        const double *vi[2] = {NULL, v};
        double *wo[1] = {W1};
        int mw = 0;
        rc = orc_phi_combo(N, swe_mv_fn, &A, 1, vi, 1, rho1, wo, &o1, &mw, NULL);
        if (rc) goto out;
    }
    for (int i = 0; i < N; i++) {
        U2[i] = u[i] + W1[i];
        e[i] = U2[i] - u[i];
    }
    orc_rhs(m, U2, D2);
    orc_jv(m, u, e, t);
    for (int i = 0; i < N; i++) {
        D2[i] = D2[i] - Fn[i] - t[i];
        a3[i] = 32.0 / 9.0 * dt * D2[i];
    }
    {
        orc_phi_opts o2 = *o;
        o2.tape = &t2;
        double rho2[1] = {1.0};
        const double *vii[4] = {NULL, v, NULL, a3};
        double *wo[1] = {W2};
        int mw = 0;
        rc = orc_phi_combo(N, swe_mv_fn, &A, 3, vii, 1, rho2, wo, &o2, &mw, NULL);
        if (rc) goto out;
    }

    /* reverse */
    memcpy(ubar_n, ubar_np1, sizeof(double) * N);
    {
        double rho2[1] = {1.0};
        const double *wb[1] = {ubar_np1};
        rc = orc_phi_adjoint(N, swe_mv_fn, &AT, swe_k_fn, &kc, kacc, &t2, 3, 1, rho2, wb, vb, o,
                             &adj[1]);
        if (rc) goto out;
    }
    for (int i = 0; i < N; i++) Dbar[i] = 32.0 / 9.0 * dt * vb[3][i];
    orc_jtv(m, U2, Dbar, Ubar2);
    orc_jtv(m, u, Dbar, t);
    for (int i = 0; i < N; i++) {
        Ubar2[i] -= t[i];
        Fbar[i] = dt * vb[1][i] - Dbar[i];
        ubar_n[i] += t[i];
    }
    orc_ktv(m, Dbar, e, t);
    for (int i = 0; i < N; i++) ubar_n[i] -= t[i];
    {
        double rho1[1] = {0.75};
        const double *wb[1] = {Ubar2};
        double *vb1[2] = {NULL, vb[1]};
        rc = orc_phi_adjoint(N, swe_mv_fn, &AT, swe_k_fn, &kc, kacc, &t1, 1, 1, rho1, wb, vb1, o,
                             &adj[0]);
        if (rc) goto out;
    }
    for (int i = 0; i < N; i++) {
        ubar_n[i] += Ubar2[i];
        Fbar[i] += dt * vb[1][i];
    }
    orc_jtv(m, u, Fbar, t);
    for (int i = 0; i < N; i++) ubar_n[i] += t[i] + kacc[i];
out:
    orc_tape_free(&t1);
    orc_tape_free(&t2);
    free(Fn); free(v); free(W1); free(W2); free(U2); free(e); free(D2); free(a3); free(t);
    free(Dbar); free(Ubar2); free(Fbar); free(kacc); free(ktmp); free(vb[1]); free(vb[3]);
    return rc;
}
