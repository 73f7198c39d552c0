/*
 * Oracle: finite-volume shallow water on the icosahedral geodesic grid.
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper gives the semi-discrete system (Sec. 2, eq. sweqsinv) in terms of
 * sparse gradient G, divergence D, vorticity V and Laplacian L matrices whose
 * entries it defers to the discretisation paper it cites.  This file writes
 * them out as the flux-form finite-volume operators on the Voronoi cells:
 *
 *   (D.F)_i   = 1/A_i sum_e l_e n_{e,i} . (F_i + F_j)/2
 *   (G psi)_i = P_i 1/A_i sum_e l_e n_{e,i} (psi_j - psi_i)/2,  P_i = I - n_i n_i^T
 *   (V.u)_i   = 1/A_i sum_e l_e t_{e,i} . (u_i + u_j)/2          (Stokes)
 *   (L psi)_i = 1/A_i sum_e (l_e/d_e) (psi_j - psi_i)
 *
 * with l_e the great-circle length of the Voronoi edge, d_e the great-circle
 * distance of the two centres, n_{e,i} the unit tangent normal at the edge
 * midpoint direction rhat_e = (x_i+x_j)/|x_i+x_j| pointing from i to j, and
 * t_{e,i} = rhat_e x n_{e,i}.
 */
#include "orc.h"
#include "orc_par.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

int orc_threads = 1;

void orc_set_threads(int nthreads) { orc_threads = nthreads > 1 ? nthreads : 1; }
int orc_get_threads(void) { return orc_threads; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* great-circle angle between unit vectors */
static double arc(const double *p, const double *q)
{
    double c[3];
    cross3(p, q, c);
    return atan2(norm3(c), dot3(p, q));
}

/* area of the spherical triangle (p,q,r) on the unit sphere
 * (Van Oosterom & Strackee 1983) */
static double sph_tri(const double *p, const double *q, const double *r)
{
    double c[3];
    cross3(q, r, c);
    double num = fabs(dot3(p, c));
    double den = 1.0 + dot3(p, q) + dot3(q, r) + dot3(r, p);
    return 2.0 * atan2(num, den);
}

int orc_swe_init(orc_swe *m, int n, const double *xyz, const int *deg, const int *nbr,
                 const double *corners, double radius, double omega, double gravity,
                 double gamma_h, double dt_e)
{
    memset(m, 0, sizeof(*m));
    m->n = n;
    m->radius = radius;
    m->omega = omega;
    m->gravity = gravity;
    m->gamma_h = gamma_h;
    m->dt_e = dt_e;
    m->xyz = malloc(sizeof(double) * 3 * n);
    m->deg = malloc(sizeof(int) * n);
    m->nbr = malloc(sizeof(int) * 6 * n);
    m->area = malloc(sizeof(double) * n);
    m->len = calloc(6 * (size_t)n, sizeof(double));
    m->dist = calloc(6 * (size_t)n, sizeof(double));
    m->nrm = calloc(18 * (size_t)n, sizeof(double));
    m->tng = calloc(18 * (size_t)n, sizeof(double));
    m->cor = malloc(sizeof(double) * n);
    m->work = malloc(sizeof(double) * 16 * (size_t)n);
    m->hs = calloc((size_t)n, sizeof(double));
    if (!m->xyz || !m->deg || !m->nbr || !m->area || !m->len || !m->dist || !m->nrm ||
        !m->tng || !m->cor || !m->work || !m->hs)
        return ORC_ENOMEM;
    memcpy(m->xyz, xyz, sizeof(double) * 3 * n);
    memcpy(m->deg, deg, sizeof(int) * n);
    memcpy(m->nbr, nbr, sizeof(int) * 6 * n);

    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *xi = xyz + 3 * i;
        int d = deg[i];
        double a = 0.0;
        for (int s = 0; s < d; s++) {
            int j = nbr[6 * i + s];
            const double *xj = xyz + 3 * j;
            const double *c0 = corners + 18 * i + 3 * ((s + d - 1) % d);
            const double *c1 = corners + 18 * i + 3 * s;
            m->len[6 * i + s] = radius * arc(c0, c1);
            m->dist[6 * i + s] = radius * arc(xi, xj);
            double r[3] = {xi[0] + xj[0], xi[1] + xj[1], xi[2] + xj[2]};
            double rn = norm3(r);
            r[0] /= rn; r[1] /= rn; r[2] /= rn;
            double dv[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
            double dr = dot3(dv, r);
            dv[0] -= dr * r[0]; dv[1] -= dr * r[1]; dv[2] -= dr * r[2];
            double dn = norm3(dv);
            double *nv = m->nrm + 18 * i + 3 * s;
            nv[0] = dv[0] / dn; nv[1] = dv[1] / dn; nv[2] = dv[2] / dn;
            cross3(r, nv, m->tng + 18 * i + 3 * s);
            a += sph_tri(xi, c0, c1);
        }
        m->area[i] = radius * radius * a;
        m->cor[i] = 2.0 * omega * xi[2];
    }
    /* eq. niu: nu = gamma_h * dxbar^4 / dt_e, dxbar = sqrt(4 pi a^2 / N_g) */
    double dx = sqrt(4.0 * M_PI * radius * radius / n);
    m->nu = gamma_h * dx * dx * dx * dx / dt_e;
    return ORC_OK;
}

void orc_swe_free(orc_swe *m)
{
    free(m->xyz); free(m->deg); free(m->nbr); free(m->area); free(m->len); free(m->dist);
    free(m->nrm); free(m->tng); free(m->cor); free(m->work); free(m->hs);
    memset(m, 0, sizeof(*m));
}

/* ------------------------------------------------------------------ */
/* operators                                                            */
/* ------------------------------------------------------------------ */
void orc_div(const orc_swe *m, const double *fx, const double *fy, const double *fz, double *out)
{
    ORC_PARFOR
    for (int i = 0; i < m->n; i++) {
        double acc = 0.0;
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *nv = m->nrm + 18 * i + 3 * s;
            double fe = nv[0] * (fx[i] + fx[j]) + nv[1] * (fy[i] + fy[j]) + nv[2] * (fz[i] + fz[j]);
            acc += m->len[6 * i + s] * fe / 2.0;
        }
        out[i] = acc / m->area[i];
    }
}

void orc_grad(const orc_swe *m, const double *psi, double *gx, double *gy, double *gz)
{
    ORC_PARFOR
    for (int i = 0; i < m->n; i++) {
        double g[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *nv = m->nrm + 18 * i + 3 * s;
            double w = m->len[6 * i + s] * (psi[j] - psi[i]) / 2.0;
            g[0] += w * nv[0]; g[1] += w * nv[1]; g[2] += w * nv[2];
        }
        g[0] /= m->area[i]; g[1] /= m->area[i]; g[2] /= m->area[i];
        const double *ni = m->xyz + 3 * i;
        double r = dot3(ni, g);
        gx[i] = g[0] - r * ni[0];
        gy[i] = g[1] - r * ni[1];
        gz[i] = g[2] - r * ni[2];
    }
}

void orc_curl(const orc_swe *m, const double *ux, const double *uy, const double *uz, double *out)
{
    ORC_PARFOR
    for (int i = 0; i < m->n; i++) {
        double acc = 0.0;
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *tv = m->tng + 18 * i + 3 * s;
            double ue = tv[0] * (ux[i] + ux[j]) + tv[1] * (uy[i] + uy[j]) + tv[2] * (uz[i] + uz[j]);
            acc += m->len[6 * i + s] * ue / 2.0;
        }
        out[i] = acc / m->area[i];
    }
}

void orc_lap(const orc_swe *m, const double *psi, double *out)
{
    ORC_PARFOR
    for (int i = 0; i < m->n; i++) {
        double acc = 0.0;
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            acc += m->len[6 * i + s] / m->dist[6 * i + s] * (psi[j] - psi[i]);
        }
        out[i] = acc / m->area[i];
    }
}

/* transposes (scatter form) */
static void div_T(const orc_swe *m, const double *w, double *rx, double *ry, double *rz)
{
    int n = m->n;
    memset(rx, 0, sizeof(double) * n);
    memset(ry, 0, sizeof(double) * n);
    memset(rz, 0, sizeof(double) * n);
    for (int i = 0; i < n; i++) {
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *nv = m->nrm + 18 * i + 3 * s;
            double c = m->len[6 * i + s] / 2.0 / m->area[i] * w[i];
            rx[i] += c * nv[0]; ry[i] += c * nv[1]; rz[i] += c * nv[2];
            rx[j] += c * nv[0]; ry[j] += c * nv[1]; rz[j] += c * nv[2];
        }
    }
}

static void grad_T(const orc_swe *m, const double *gx, const double *gy, const double *gz, double *out)
{
    int n = m->n;
    memset(out, 0, sizeof(double) * n);
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        double g[3] = {gx[i], gy[i], gz[i]};
        double r = dot3(ni, g);
        double pg[3] = {g[0] - r * ni[0], g[1] - r * ni[1], g[2] - r * ni[2]};
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *nv = m->nrm + 18 * i + 3 * s;
            double c = m->len[6 * i + s] / 2.0 / m->area[i] * dot3(nv, pg);
            out[j] += c;
            out[i] -= c;
        }
    }
}

static void curl_T(const orc_swe *m, const double *w, double *rx, double *ry, double *rz)
{
    int n = m->n;
    memset(rx, 0, sizeof(double) * n);
    memset(ry, 0, sizeof(double) * n);
    memset(rz, 0, sizeof(double) * n);
    for (int i = 0; i < n; i++) {
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            const double *tv = m->tng + 18 * i + 3 * s;
            double c = m->len[6 * i + s] / 2.0 / m->area[i] * w[i];
            rx[i] += c * tv[0]; ry[i] += c * tv[1]; rz[i] += c * tv[2];
            rx[j] += c * tv[0]; ry[j] += c * tv[1]; rz[j] += c * tv[2];
        }
    }
}

static void lap_T(const orc_swe *m, const double *w, double *out)
{
    int n = m->n;
    memset(out, 0, sizeof(double) * n);
    for (int i = 0; i < n; i++) {
        for (int s = 0; s < m->deg[i]; s++) {
            int j = m->nbr[6 * i + s];
            double c = m->len[6 * i + s] / m->dist[6 * i + s] / m->area[i] * w[i];
            out[j] += c;
            out[i] -= c;
        }
    }
}

/* ------------------------------------------------------------------ */
/* right-hand side, eq. sweqsinv plus D_f = -nu L^2 on every variable   */
/* ------------------------------------------------------------------ */
void orc_rhs(const orc_swe *m, const double *u, double *f)
{
    int n = m->n;
    const double *ux = u, *uy = u + n, *uz = u + 2 * n, *h = u + 3 * n;
    double *E = m->work, *eta = m->work + n, *gx = m->work + 2 * n, *gy = m->work + 3 * n,
           *gz = m->work + 4 * n, *l1 = m->work + 5 * n, *l2 = m->work + 6 * n,
           *hx = m->work + 7 * n, *hy = m->work + 8 * n, *hz = m->work + 9 * n;
    double g = m->gravity;
    /* total energy  E = |u|^2/2 + g (h + h_s) */
    ORC_PARFOR
    for (int i = 0; i < n; i++)
        E[i] = (ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i]) / 2.0 + g * (h[i] + m->hs[i]);
    /* absolute vorticity eta = V.u + f (eq. vort) */
    orc_curl(m, ux, uy, uz, eta);
    ORC_PARFOR
    for (int i = 0; i < n; i++) eta[i] += m->cor[i];
    orc_grad(m, E, gx, gy, gz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        double Px = ni[1] * uz[i] - ni[2] * uy[i];
        double Py = ni[2] * ux[i] - ni[0] * uz[i];
        double Pz = ni[0] * uy[i] - ni[1] * ux[i];
        f[i] = -eta[i] * Px - gx[i];
        f[n + i] = -eta[i] * Py - gy[i];
        f[2 * n + i] = -eta[i] * Pz - gz[i];
    }
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        hx[i] = ux[i] * h[i];
        hy[i] = uy[i] * h[i];
        hz[i] = uz[i] * h[i];
    }
    orc_div(m, hx, hy, hz, f + 3 * n);
    ORC_PARFOR
    for (int i = 0; i < n; i++) f[3 * n + i] = -f[3 * n + i];
    /* dissipation D_f psi = -nu L(L psi) for each prognostic variable */
    for (int c = 0; c < 4; c++) {
        orc_lap(m, u + c * n, l1);
        orc_lap(m, l1, l2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) f[c * n + i] -= m->nu * l2[i];
    }
}

/* ------------------------------------------------------------------ */
/* J(u) v = J_v v + J_r v + J_m v  (eqs. dynjs-dynjc)                   */
/* ------------------------------------------------------------------ */
void orc_jv(const orc_swe *m, const double *u, const double *v, double *out)
{
    int n = m->n;
    const double *ux = u, *uy = u + n, *uz = u + 2 * n, *h = u + 3 * n;
    const double *vx = v, *vy = v + n, *vz = v + 2 * n, *vh = v + 3 * n;
    double *eta = m->work, *zv = m->work + n, *s = m->work + 2 * n, *gx = m->work + 3 * n,
           *gy = m->work + 4 * n, *gz = m->work + 5 * n, *l1 = m->work + 6 * n,
           *l2 = m->work + 7 * n, *fx = m->work + 8 * n, *fy = m->work + 9 * n,
           *fz = m->work + 10 * n, *dv = m->work + 11 * n;
    double g = m->gravity;
    orc_curl(m, ux, uy, uz, eta);
    ORC_PARFOR
    for (int i = 0; i < n; i++) eta[i] += m->cor[i];

    /* J_v v: -P^i (V v)_i in each velocity row */
    orc_curl(m, vx, vy, vz, zv);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        double Px = ni[1] * uz[i] - ni[2] * uy[i];
        double Py = ni[2] * ux[i] - ni[0] * uz[i];
        double Pz = ni[0] * uy[i] - ni[1] * ux[i];
        out[i] = -Px * zv[i];
        out[n + i] = -Py * zv[i];
        out[2 * n + i] = -Pz * zv[i];
        out[3 * n + i] = 0.0;
    }
    /* J_r v: rotation rows (row 2 with the signs of d(-eta P_y)/du) */
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        out[i] += eta[i] * ni[2] * vy[i] - eta[i] * ni[1] * vz[i];
        out[n + i] += -eta[i] * ni[2] * vx[i] + eta[i] * ni[0] * vz[i];
        out[2 * n + i] += eta[i] * ni[1] * vx[i] - eta[i] * ni[0] * vy[i];
    }
    /* J_r v: dissipation D_f = -nu L^2 on the diagonal blocks */
    for (int c = 0; c < 4; c++) {
        orc_lap(m, v + c * n, l1);
        orc_lap(m, l1, l2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) out[c * n + i] -= m->nu * l2[i];
    }
    /* J_m v: velocity rows -G (u . v_vel + g v_h) */
    ORC_PARFOR
    for (int i = 0; i < n; i++) s[i] = ux[i] * vx[i] + uy[i] * vy[i] + uz[i] * vz[i] + g * vh[i];
    orc_grad(m, s, gx, gy, gz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] -= gx[i];
        out[n + i] -= gy[i];
        out[2 * n + i] -= gz[i];
    }
    /* J_m v: height row -D.(h v_vel) - D.(u v_h) */
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        fx[i] = h[i] * vx[i] + ux[i] * vh[i];
        fy[i] = h[i] * vy[i] + uy[i] * vh[i];
        fz[i] = h[i] * vz[i] + uz[i] * vh[i];
    }
    orc_div(m, fx, fy, fz, dv);
    ORC_PARFOR
    for (int i = 0; i < n; i++) out[3 * n + i] -= dv[i];
}

/* J(u)^T w, the Euclidean transpose of orc_jv */
void orc_jtv(const orc_swe *m, const double *u, const double *w, double *out)
{
    int n = m->n;
    const double *ux = u, *uy = u + n, *uz = u + 2 * n, *h = u + 3 * n;
    const double *wx = w, *wy = w + n, *wz = w + 2 * n, *wh = w + 3 * n;
    double *eta = m->work, *a = m->work + n, *rx = m->work + 2 * n, *ry = m->work + 3 * n,
           *rz = m->work + 4 * n, *q = m->work + 5 * n, *l1 = m->work + 6 * n,
           *l2 = m->work + 7 * n, *dx = m->work + 8 * n, *dy = m->work + 9 * n,
           *dz = m->work + 10 * n;
    double g = m->gravity;
    orc_curl(m, ux, uy, uz, eta);
    ORC_PARFOR
    for (int i = 0; i < n; i++) eta[i] += m->cor[i];

    /* (J_v)^T: -V^T (w_vel . P) */
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        double Px = ni[1] * uz[i] - ni[2] * uy[i];
        double Py = ni[2] * ux[i] - ni[0] * uz[i];
        double Pz = ni[0] * uy[i] - ni[1] * ux[i];
        a[i] = wx[i] * Px + wy[i] * Py + wz[i] * Pz;
    }
    curl_T(m, a, rx, ry, rz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] = -rx[i];
        out[n + i] = -ry[i];
        out[2 * n + i] = -rz[i];
        out[3 * n + i] = 0.0;
    }
    /* (J_r)^T rotation: transpose of the 3x3 per-cell block */
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        out[i] += -eta[i] * ni[2] * wy[i] + eta[i] * ni[1] * wz[i];
        out[n + i] += eta[i] * ni[2] * wx[i] - eta[i] * ni[0] * wz[i];
        out[2 * n + i] += -eta[i] * ni[1] * wx[i] + eta[i] * ni[0] * wy[i];
    }
    /* (J_r)^T dissipation: -nu (L^T)^2 */
    for (int c = 0; c < 4; c++) {
        lap_T(m, w + c * n, l1);
        lap_T(m, l1, l2);
        ORC_PARFOR
        for (int i = 0; i < n; i++) out[c * n + i] -= m->nu * l2[i];
    }
    /* (J_m)^T velocity rows: q = G^T w_vel; v_vel gets -q u, v_h gets -g q */
    grad_T(m, wx, wy, wz, q);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] -= q[i] * ux[i];
        out[n + i] -= q[i] * uy[i];
        out[2 * n + i] -= q[i] * uz[i];
        out[3 * n + i] -= g * q[i];
    }
    /* (J_m)^T height row: r = D^T w_h; v_vel gets -h r, v_h gets -r . u */
    div_T(m, wh, dx, dy, dz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] -= h[i] * dx[i];
        out[n + i] -= h[i] * dy[i];
        out[2 * n + i] -= h[i] * dz[i];
        out[3 * n + i] -= dx[i] * ux[i] + dy[i] * uy[i] + dz[i] * uz[i];
    }
}

/* K(a, b) = grad_u <a, J(u) b>.  F is quadratic, so J(u) is affine in u and
 * K does not depend on u: <d, K(a, b)> = <a, (J(d) - J(0)) b>.  The terms of
 * J(u) b that move with u are
 *   J_v:  -(V b_vel)(n x u)            -> -(V b)_i (a_i x n_i)
 *   J_r:  (V u)(b_vel x n)  (eta = V u + f) -> V^T c,  c_i = a_i . (b_i x n_i)
 *   J_m:  -G(u . b_vel)                -> -(G^T a_vel)_i b_i
 *         -D.(h b_vel + b_h u)         -> r = D^T a_h: h gets -r_i . b_i,
 *                                         velocity gets -b_h,i r_i
 * (the dissipation does not depend on u). */
void orc_ktv(const orc_swe *m, const double *a, const double *b, double *out)
{
    int n = m->n;
    const double *ax = a, *ay = a + n, *az = a + 2 * n, *ah = a + 3 * n;
    const double *bx = b, *by = b + n, *bz = b + 2 * n, *bh = b + 3 * n;
    double *zb = m->work, *c = m->work + n, *rx = m->work + 2 * n, *ry = m->work + 3 * n,
           *rz = m->work + 4 * n, *q = m->work + 5 * n, *dx = m->work + 6 * n,
           *dy = m->work + 7 * n, *dz = m->work + 8 * n;
    orc_curl(m, bx, by, bz, zb);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        const double *ni = m->xyz + 3 * i;
        /* a x n */
        double cx = ay[i] * ni[2] - az[i] * ni[1];
        double cy = az[i] * ni[0] - ax[i] * ni[2];
        double cz = ax[i] * ni[1] - ay[i] * ni[0];
        out[i] = -zb[i] * cx;
        out[n + i] = -zb[i] * cy;
        out[2 * n + i] = -zb[i] * cz;
        out[3 * n + i] = 0.0;
        /* b x n */
        double ex = by[i] * ni[2] - bz[i] * ni[1];
        double ey = bz[i] * ni[0] - bx[i] * ni[2];
        double ez = bx[i] * ni[1] - by[i] * ni[0];
        c[i] = ax[i] * ex + ay[i] * ey + az[i] * ez;
    }
    curl_T(m, c, rx, ry, rz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] += rx[i];
        out[n + i] += ry[i];
        out[2 * n + i] += rz[i];
    }
    grad_T(m, ax, ay, az, q);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] -= q[i] * bx[i];
        out[n + i] -= q[i] * by[i];
        out[2 * n + i] -= q[i] * bz[i];
    }
    div_T(m, ah, dx, dy, dz);
    ORC_PARFOR
    for (int i = 0; i < n; i++) {
        out[i] -= bh[i] * dx[i];
        out[n + i] -= bh[i] * dy[i];
        out[2 * n + i] -= bh[i] * dz[i];
        out[3 * n + i] -= dx[i] * bx[i] + dy[i] * by[i] + dz[i] * bz[i];
    }
}

/* ------------------------------------------------------------------ */
static void swe_rhs_cb(void *ctx, const double *u, double *f) { orc_rhs((const orc_swe *)ctx, u, f); }
static void swe_jv_cb(void *ctx, const double *u, const double *v, double *o)
{
    orc_jv((const orc_swe *)ctx, u, v, o);
}

void orc_swe_problem(orc_swe *m, orc_problem *pb)
{
    pb->n = 4 * m->n;
    pb->rhs = swe_rhs_cb;
    pb->jv = swe_jv_cb;
    pb->ctx = m;
}

void orc_diagnostics(const orc_swe *m, const double *u, double out[3])
{
    int n = m->n;
    const double *ux = u, *uy = u + n, *uz = u + 2 * n, *h = u + 3 * n;
    double *zeta = m->work;
    orc_curl(m, ux, uy, uz, zeta);
    double mass = 0.0, energy = 0.0, enstrophy = 0.0;
    for (int i = 0; i < n; i++) {
        double a = m->area[i];
        double speed2 = ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i];
        double absvort = zeta[i] + m->cor[i];
        mass += a * h[i];
        energy += a * (h[i] * speed2 / 2.0 + m->gravity * h[i] * h[i] / 2.0 +
                       m->gravity * h[i] * m->hs[i]);
        enstrophy += a * absvort * absvort / (2.0 * h[i]);
    }
    out[0] = mass;
    out[1] = energy;
    out[2] = enstrophy;
}

void orc_swe_set_topography(orc_swe *m, const double *hs)
{
    for (int i = 0; i < m->n; i++) m->hs[i] = hs ? hs[i] : 0.0;
}
