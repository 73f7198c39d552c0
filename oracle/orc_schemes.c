/*
 * Oracle: exponential Rosenbrock schemes.  TEST INFRASTRUCTURE ONLY.
 *
 * With A = dt J_n and v = dt F(u_n) (Sec. 4.4), each scheme is a short
 * sequence of phipm_simul_iom2 calls whose outputs carry the rho_i^l factor
 * (W_i = sum_l rho_i^l phi_l(rho_i A) v_l):
 *
 *   exprb42  (eq. 3.11): (i)  rho = [3/4], v_1 = v              -> U2 = u_n + W
 *                        (ii) rho = [1], v_1 = v, v_3 = 32/9 dt D2 -> u_{n+1} = u_n + W
 *   pexprb43 (eq. 3.12): (i)  rho = [1/2, 1], v_1 = v           -> U2, U3 = u_n + W_1, u_n + W_2
 *                        (ii) rho = [1], v_3 = dt(16 D2 - 2 D3), v_4 = dt(-48 D2 + 12 D3)
 *                             -> u_{n+1} = U3 + W
 *   exprb53  (eq. 3.13): (i)  rho = [1/2, 9/10], v_1 = v        -> U2 = u_n + W_1
 *                        (ii) rho = [1/2, 9/10], v_3 = dt D2
 *                             -> U3 = u_n + W(i)_2 + 27/25*8 W(ii)_1 + 729/125*(10/9)^3 W(ii)_2
 *                        (iii) rho = [1], v_1 = v, v_3 = dt(18 D2 - 250/81 D3),
 *                              v_4 = dt(-60 D2 + 500/27 D3)  -> u_{n+1} = u_n + W
 *   epi3     (eq. epi3): rho = [1], v_1 = v, v_2 = 2/3 dt R_{n-1},
 *                        R_{n-1} = F(u_{n-1}) - F(u_n) - J_n (u_{n-1} - u_n);
 *                        first step EPI2 (eq. 3.5): rho = [1], v_1 = v.
 *   EPI2     (eq. 3.5):  rho = [1], v_1 = v.
 *   exprb42m (eq. 3.11 with the two phi_1 evaluations in one call, the
 *             variant Sec. 4.4's mapping leaves open; the phi-combination is
 *             linear in v_1..v_p, so call (ii) keeps only its v_3 part):
 *                        (i)  rho = [3/4, 1], v_1 = v  -> U2 = u_n + W_1, W_2 = phi_1(A) v
 *                        (ii) rho = [1], v_3 = 32/9 dt D2 -> u_{n+1} = u_n + W_2 + W
 *
 *   exprb32  (a third-order scheme of the form eq. 3.10 with c_2 = 1 and
 *             b_2 = 2 phi_3, the solution of Table 1's condition 1; not one
 *             of the paper's schemes, used to check the tableau driver):
 *                        (i)  rho = [1], v_1 = v          -> U2 = u_n + W
 *                        (ii) rho = [1], v_3 = 2 dt D2    -> u_{n+1} = U2 + W
 *
 * D_i = N_n(U_i) - N_n(u_n) = F(U_i) - F(u_n) - J_n (U_i - u_n) (eq. Dni).
 * The rescaling factors of exprb53's U3 convert the rho^l-weighted outputs
 * back to the plain phi_3 terms of eq. 3.13 (coefficient 729/125).
 */
#include "orc.h"
#include "orc_par.h"
#include <stdlib.h>
#include <string.h>

typedef struct { const orc_problem *pb; const double *u; double dt; } jmv_ctx;

static void jmv(void *ctx, const double *x, double *y)
{
    const jmv_ctx *c = ctx;
    c->pb->jv(c->pb->ctx, c->u, x, y);
    int n = c->pb->n;
    ORC_PARFOR
    for (int i = 0; i < n; i++) y[i] *= c->dt;
}

int orc_step_state_init(orc_step_state *s, int n)
{
    memset(s, 0, sizeof(*s));
    s->u_prev = calloc(n, sizeof(double));
    s->f_prev = calloc(n, sizeof(double));
    return (s->u_prev && s->f_prev) ? ORC_OK : ORC_ENOMEM;
}

void orc_step_state_free(orc_step_state *s)
{
    free(s->u_prev);
    free(s->f_prev);
    memset(s, 0, sizeof(*s));
}

/* D = F(U) - Fn - J_n (U - u_n) */
static void nonlin_diff(const orc_problem *pb, const double *un, const double *Fn,
                        const double *U, double *D, double *t1, double *t2)
{
    int n = pb->n;
    pb->rhs(pb->ctx, U, D);
    ORC_PARFOR
    for (int i = 0; i < n; i++) t1[i] = U[i] - un[i];
    pb->jv(pb->ctx, un, t1, t2);
    ORC_PARFOR
    for (int i = 0; i < n; i++) D[i] = D[i] - Fn[i] - t2[i];
}

int orc_step(const orc_problem *pb, int method, double *u, double dt, orc_step_state *s,
             const orc_phi_opts *o)
{
    int n = pb->n;
    int rc = ORC_OK;
    double *Fn = calloc(n, sizeof(double)), *v = calloc(n, sizeof(double));
    double *W1 = calloc(n, sizeof(double)), *W2 = calloc(n, sizeof(double));
    double *X1 = calloc(n, sizeof(double)), *X2 = calloc(n, sizeof(double));
    double *U2 = calloc(n, sizeof(double)), *U3 = calloc(n, sizeof(double));
    double *D2 = calloc(n, sizeof(double)), *D3 = calloc(n, sizeof(double));
    double *a3 = calloc(n, sizeof(double)), *a4 = calloc(n, sizeof(double));
    double *t1 = calloc(n, sizeof(double)), *t2 = calloc(n, sizeof(double));
    if (!Fn || !v || !W1 || !W2 || !X1 || !X2 || !U2 || !U3 || !D2 || !D3 || !a3 || !a4 ||
        !t1 || !t2) { rc = ORC_ENOMEM; goto out; }

    jmv_ctx jc = {pb, u, dt};
    pb->rhs(pb->ctx, u, Fn);
    ORC_PARFOR
    for (int i = 0; i < n; i++) v[i] = dt * Fn[i];

    if (method == ORC_EXPRB42) {
        double rho1[1] = {0.75}, rho2[1] = {1.0};
        const double *vi[2] = {NULL, v};
        double *wo[1] = {W1};
        rc = orc_phi_combo(n, jmv, &jc, 1, vi, 1, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) U2[i] = u[i] + W1[i];
        nonlin_diff(pb, u, Fn, U2, D2, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) a3[i] = 32.0 / 9.0 * dt * D2[i];
        const double *vii[4] = {NULL, v, NULL, a3};
        double *wo2[1] = {W2};
        rc = orc_phi_combo(n, jmv, &jc, 3, vii, 1, rho2, wo2, o, &s->m_warm[1], &s->calls[1]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = u[i] + W2[i];
    } else if (method == ORC_EXPRB42M) {
        double rho1[2] = {0.75, 1.0}, rho2[1] = {1.0};
        const double *vi[2] = {NULL, v};
        double *wo[2] = {W1, X1};
        rc = orc_phi_combo(n, jmv, &jc, 1, vi, 2, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) U2[i] = u[i] + W1[i];
        nonlin_diff(pb, u, Fn, U2, D2, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) a3[i] = 32.0 / 9.0 * dt * D2[i];
        const double *vii[4] = {NULL, NULL, NULL, a3};
        double *wo2[1] = {W2};
        rc = orc_phi_combo(n, jmv, &jc, 3, vii, 1, rho2, wo2, o, &s->m_warm[1], &s->calls[1]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = u[i] + X1[i] + W2[i];
    } else if (method == ORC_PEXPRB43) {
        double rho1[2] = {0.5, 1.0}, rho2[1] = {1.0};
        const double *vi[2] = {NULL, v};
        double *wo[2] = {W1, W2};
        rc = orc_phi_combo(n, jmv, &jc, 1, vi, 2, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) {
            U2[i] = u[i] + W1[i];
            U3[i] = u[i] + W2[i];
        }
        nonlin_diff(pb, u, Fn, U2, D2, t1, t2);
        nonlin_diff(pb, u, Fn, U3, D3, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) {
            a3[i] = dt * (16.0 * D2[i] - 2.0 * D3[i]);
            a4[i] = dt * (-48.0 * D2[i] + 12.0 * D3[i]);
        }
        const double *vii[5] = {NULL, NULL, NULL, a3, a4};
        double *wo2[1] = {X1};
        rc = orc_phi_combo(n, jmv, &jc, 4, vii, 1, rho2, wo2, o, &s->m_warm[1], &s->calls[1]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = U3[i] + X1[i];
    } else if (method == ORC_EXPRB53) {
        double rho1[2] = {0.5, 0.9}, rho3[1] = {1.0};
        const double *vi[2] = {NULL, v};
        double *wo[2] = {W1, W2};
        rc = orc_phi_combo(n, jmv, &jc, 1, vi, 2, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) U2[i] = u[i] + W1[i];
        nonlin_diff(pb, u, Fn, U2, D2, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) a3[i] = dt * D2[i];
        const double *vii[4] = {NULL, NULL, NULL, a3};
        double *wo2[2] = {X1, X2};
        rc = orc_phi_combo(n, jmv, &jc, 3, vii, 2, rho1, wo2, o, &s->m_warm[1], &s->calls[1]);
        if (rc) goto out;
        /* 27/25 phi_3(Z/2) D2 = 27/25 * 2^3 * W(ii)_1 ; 729/125 phi_3(9Z/10) D2 =
         * 729/125 * (10/9)^3 * W(ii)_2 = 8 W(ii)_2 */
        ORC_PARFOR
        for (int i = 0; i < n; i++) U3[i] = u[i] + W2[i] + 216.0 / 25.0 * X1[i] + 8.0 * X2[i];
        nonlin_diff(pb, u, Fn, U3, D3, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) {
            a3[i] = dt * (18.0 * D2[i] - 250.0 / 81.0 * D3[i]);
            a4[i] = dt * (-60.0 * D2[i] + 500.0 / 27.0 * D3[i]);
        }
        const double *viii[5] = {NULL, v, NULL, a3, a4};
        double *wo3[1] = {W1};
        rc = orc_phi_combo(n, jmv, &jc, 4, viii, 1, rho3, wo3, o, &s->m_warm[2], &s->calls[2]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = u[i] + W1[i];
    } else if (method == ORC_EXPRB32) {
        double rho1[1] = {1.0};
        const double *vi[2] = {NULL, v};
        double *wo[1] = {W1};
        rc = orc_phi_combo(n, jmv, &jc, 1, vi, 1, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) U2[i] = u[i] + W1[i];
        nonlin_diff(pb, u, Fn, U2, D2, t1, t2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) a3[i] = 2.0 * dt * D2[i];
        const double *vii[4] = {NULL, NULL, NULL, a3};
        double *wo2[1] = {W2};
        rc = orc_phi_combo(n, jmv, &jc, 3, vii, 1, rho1, wo2, o, &s->m_warm[1], &s->calls[1]);
        if (rc) goto out;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = U2[i] + W2[i];
    } else if (method == ORC_EPI3 || method == ORC_EPI2) {
        double rho1[1] = {1.0};
        if (method == ORC_EPI3 && s->have_prev) {
            /* R_{n-1} = F(u_{n-1}) - F(u_n) - J_n (u_{n-1} - u_n) */
            ORC_PARFOR
            for (int i = 0; i < n; i++) t1[i] = s->u_prev[i] - u[i];
            pb->jv(pb->ctx, u, t1, t2);
            ORC_PARFOR
            for (int i = 0; i < n; i++) a3[i] = 2.0 / 3.0 * dt * (s->f_prev[i] - Fn[i] - t2[i]);
            const double *vi[3] = {NULL, v, a3};
            double *wo[1] = {W1};
            rc = orc_phi_combo(n, jmv, &jc, 2, vi, 1, rho1, wo, o, &s->m_warm[0], &s->calls[0]);
        } else {
            const double *vi[2] = {NULL, v};
            double *wo[1] = {W1};
            rc = orc_phi_combo(n, jmv, &jc, 1, vi, 1, rho1, wo, o, &s->m_warm[1], &s->calls[1]);
        }
        if (rc) goto out;
        memcpy(s->u_prev, u, sizeof(double) * n);
        memcpy(s->f_prev, Fn, sizeof(double) * n);
        s->have_prev = 1;
        ORC_PARFOR
        for (int i = 0; i < n; i++) u[i] = u[i] + W1[i];
    } else {
        rc = ORC_EINVAL;
    }
out:
    free(Fn); free(v); free(W1); free(W2); free(X1); free(X2); free(U2); free(U3);
    free(D2); free(D3); free(a3); free(a4); free(t1); free(t2);
    return rc;
}
