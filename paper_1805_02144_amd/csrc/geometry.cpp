// Host-side preparation of the finite-volume stencil weights (Sec. 2).
//
// The paper writes the semi-discrete model with sparse gradient, divergence,
// vorticity and Laplacian matrices on the Voronoi cells of the icosahedral
// grid.  The flux-form operators use, per edge e from cell i to j,
//   a_s = l_e n_e / (2 A_i)   (flux divergence: sum_s a_s . (F_i + F_j);
//                              gradient: P_i sum_s a_s (psi_j - psi_i))
//   b_s = l_e t_e / (2 A_i)   (circulation: sum_s b_s . (u_i + u_j))
//   c_s = l_e / (d_e A_i)     (Laplacian: sum_s c_s (psi_j - psi_i))
// with l_e the great-circle length of the Voronoi edge (between the two
// corners that bound it), d_e the great-circle distance of the centres,
// A_i the spherical area of the cell, n_e the unit tangent normal at the
// edge direction rhat_e = (x_i + x_j)/|x_i + x_j| pointing from i to j, and
// t_e = rhat_e x n_e.  On the unit sphere x_j - x_i is orthogonal to
// x_i + x_j, so n_e = (x_j - x_i)/|x_j - x_i| and t_e = 2 (x_i x x_j) /
// (|x_i + x_j| |x_j - x_i|): the kernels rebuild a_s and b_s from two
// scalars per edge and the centres they already load,
//   alpha_s = l_e / (2 A_i |x_j - x_i|),  beta_s = 2 alpha_s / |x_i + x_j|,
// of which alpha_s is stored and beta_s formed in the kernels (the
// LDS-staged product forms alpha_s as well, as c_s (a / 2) asin(y) / y with
// the chord 2y = |x_j - x_i|, since d_e = 2 a asin(y)).  Pentagon slot 5
// gets zero weights.
//
// For the LDS-staged product of large grids, build_halo cuts the cells into
// chunks of kChunk consecutive cells and lists each chunk's one-ring halo.
#include <algorithm>
#include <cmath>

#include "xrb_internal.h"

namespace xrb {
namespace {

// the range of the kernels' asin series (kAsinY2Max in stencil_common.h)
constexpr double kAsinY2MaxHost = 0.01;

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double len(V3 a) { return std::sqrt(dot(a, a)); }
// angle between two unit vectors
inline double angle(V3 a, V3 b) { return std::atan2(len(cross(a, b)), dot(a, b)); }
// spherical excess of the unit-sphere triangle (a, b, c)
inline double excess(V3 a, V3 b, V3 c) {
    double num = std::fabs(dot(a, cross(b, c)));
    double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
    return 2.0 * std::atan2(num, den);
}

}  // namespace

int build_geometry(const xrb_mesh &mesh, const xrb_params &prm, HostGeometry &geo,
                   std::string &err) {
    const int64_t n = mesh.n_cells;
    if (n < 12 || !mesh.xyz || !mesh.deg || !mesh.nbr || !mesh.corners) {
        err = "mesh: null array or fewer than 12 cells";
        return XRB_EINVAL;
    }
    if (n > (int64_t)1 << 28) {
        err = "mesh: too many cells";
        return XRB_EINVAL;
    }
    const double R = prm.radius;
    geo.n = (int)n;
    auto resize6 = [&](std::vector<double> &v) { v.assign(6 * (size_t)n, 0.0); };
    geo.nbr.assign(6 * (size_t)n, 0);
    resize6(geo.alpha); resize6(geo.cl);
    geo.cen.assign(4 * (size_t)n, 0.0);
    geo.area.assign((size_t)n, 0.0);

    auto X = [&](int64_t i) { return V3{mesh.xyz[3 * i], mesh.xyz[3 * i + 1], mesh.xyz[3 * i + 2]}; };
    auto CRN = [&](int64_t i, int s) {
        const double *c = mesh.corners + 18 * i + 3 * s;
        return V3{c[0], c[1], c[2]};
    };

    for (int64_t i = 0; i < n; ++i) {
        const int d = mesh.deg[i];
        if (d != 5 && d != 6) {
            err = "mesh: degree must be 5 or 6";
            return XRB_EINVAL;
        }
        const V3 xi = X(i);
        // cell area first (needed by every weight)
        double ex = 0.0;
        for (int s = 0; s < d; ++s) ex += excess(xi, CRN(i, (s + d - 1) % d), CRN(i, s));
        const double area = R * R * ex;
        for (int s = 0; s < 6; ++s) {
            const size_t k = 6 * (size_t)i + s;     // cell-major: the 6 slots of a cell are contiguous
            if (s >= d) {                      // pentagon padding: self, zero weights
                geo.nbr[k] = (int32_t)i;
                continue;
            }
            const int32_t j = mesh.nbr[6 * i + s];
            if (j < 0 || j >= n || j == i) {
                err = "mesh: neighbour index out of range";
                return XRB_EINVAL;
            }
            geo.nbr[k] = j;
            const V3 xj = X(j);
            const double le = R * angle(CRN(i, (s + d - 1) % d), CRN(i, s));
            const double de = R * angle(xi, xj);
            const double chord = len(sub(xj, xi));
            geo.alpha[k] = le / (2.0 * area * chord);
            geo.cl[k] = le / (de * area);
        }
        double *ce = &geo.cen[4 * (size_t)i];
        ce[0] = xi.x; ce[1] = xi.y; ce[2] = xi.z;
        ce[3] = 1.0 / area;
        geo.area[i] = area;
    }
    const double dxbar = std::sqrt(4.0 * M_PI * R * R / (double)n);
    geo.nu = prm.gamma_h * dxbar * dxbar * dxbar * dxbar / prm.dt_e;
    return XRB_OK;
}

void build_halo(HostGeometry &geo) {
    geo.hoff.clear();
    geo.hids.clear();
    geo.lnbr.clear();
    const int n = geo.n;
    const int nch = (n + kChunk - 1) / kChunk;
    std::vector<int32_t> hoff(nch + 1, 0), hids;
    std::vector<uint16_t> lnbr(6 * (size_t)n, 0);
    // the product's alpha series holds for half-chords y with y^2 <= kAsinY2MaxHost
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < 6; ++s) {
            const int j = geo.nbr[6 * (size_t)i + s];
            double y2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double dx = geo.cen[4 * (size_t)j + c] - geo.cen[4 * (size_t)i + c];
                y2 += 0.25 * dx * dx;
            }
            if (y2 > kAsinY2MaxHost) return;   // tables stay empty: the product keeps its gathers
        }
    std::vector<int32_t> ring;
    for (int k = 0; k < nch; ++k) {
        const int c0 = k * kChunk, c1 = std::min(n, c0 + kChunk);
        ring.clear();
        for (int i = c0; i < c1; ++i)
            for (int s = 0; s < 6; ++s) {
                const int j = geo.nbr[6 * (size_t)i + s];
                if (j < c0 || j >= c1) ring.push_back(j);
            }
        std::sort(ring.begin(), ring.end());
        ring.erase(std::unique(ring.begin(), ring.end()), ring.end());
        if ((int)ring.size() > kHaloMax) return;   // tables stay empty: the product keeps its gathers
        for (int i = c0; i < c1; ++i)
            for (int s = 0; s < 6; ++s) {
                const int j = geo.nbr[6 * (size_t)i + s];
                const int lj = (j >= c0 && j < c1)
                                   ? j - c0
                                   : kChunk + (int)(std::lower_bound(ring.begin(), ring.end(), j) - ring.begin());
                lnbr[6 * (size_t)i + s] = (uint16_t)lj;
            }
        hids.insert(hids.end(), ring.begin(), ring.end());
        hoff[k + 1] = (int32_t)hids.size();
    }
    geo.hoff.swap(hoff);
    geo.hids.swap(hids);
    geo.lnbr.swap(lnbr);
}

}  // namespace xrb
