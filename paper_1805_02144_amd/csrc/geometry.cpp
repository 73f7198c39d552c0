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
// LDS-staged product forms both from c_s and the chord 2y = |x_j - x_i|:
// alpha_s = c_s (a / 2) asin(y) / y since d_e = 2 a asin(y), and
// beta_s = alpha_s (1 - y^2)^(-1/2) since |x_i + x_j|^2 = 4 - 4 y^2).
// Pentagon slot 5 gets zero weights.
//
// The kernels number the cells in an order of their own: the caller's cell
// i sits at position inv(i) of every internal vector, with perm(p) = i.
// The order is a recursive coordinate bisection of the centres: a set of
// cells is split across the coordinate axis of its widest extent, the first
// part holding a whole number of kChunk-cell chunks (the nearest to half),
// until a part fits one chunk; each chunk keeps its cells in the caller's
// order.  Consecutive chunks are then compact, neighbouring patches, so a
// chunk's one-ring halo is close to a patch's perimeter (about 72 cells
// per 256 on the icosahedral grids, against 120 for the subdivision's own
// numbering), and the cells an XCD sweeps form one region of the sphere.
//
// For the LDS-staged product of large grids, build_halo cuts the cells into
// chunks of kChunk consecutive cells and lists each chunk's one-ring halo.
#include <algorithm>
#include <numeric>
#include <cmath>

#include "xrb_internal.h"

namespace xrb {
namespace {

// the range of the LDS-staged product's weight series (kShortY2Max in
// stencil_common.h), and of its four-term form (kShort4Y2Max)
constexpr double kShortY2MaxHost = 4e-4;
constexpr double kShort4Y2MaxHost = 3e-5;

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

// Recursive coordinate bisection of cells idx[0, cnt) into chunks (see the
// top of this file); the explicit stack keeps the depth off the call stack.
void bisect_cells(const double *xyz, int32_t *idx, int64_t cnt) {
    struct Part {
        int64_t lo, cnt;
    };
    std::vector<Part> todo{{0, cnt}};
    while (!todo.empty()) {
        const Part pt = todo.back();
        todo.pop_back();
        int32_t *a = idx + pt.lo;
        if (pt.cnt <= kChunk) {
            std::sort(a, a + pt.cnt);
            continue;
        }
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t k = 0; k < pt.cnt; ++k)
            for (int c = 0; c < 3; ++c) {
                const double v = xyz[3 * (int64_t)a[k] + c];
                lo[c] = std::min(lo[c], v);
                hi[c] = std::max(hi[c], v);
            }
        int ax = 0;
        for (int c = 1; c < 3; ++c)
            if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
        // first part: whole chunks, the nearest count to half (at least one)
        int64_t nl = (pt.cnt / 2 + kChunk / 2) / kChunk * kChunk;
        nl = std::max<int64_t>(kChunk, std::min(nl, pt.cnt - 1));
        // split at the nl-th centre along the axis (ties by cell number)
        std::nth_element(a, a + nl, a + pt.cnt, [&](int32_t p, int32_t q) {
            const double vp = xyz[3 * (int64_t)p + ax], vq = xyz[3 * (int64_t)q + ax];
            return vp < vq || (vp == vq && p < q);
        });
        todo.push_back({pt.lo + nl, pt.cnt - nl});
        todo.push_back({pt.lo, nl});
    }
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
    for (int64_t i = 0; i < n; ++i)
        for (int s = 0; s < 6; ++s) {
            const int32_t j = mesh.nbr[6 * i + s];
            if (j < 0 || j >= n) {
                err = "mesh: neighbour index out of range";
                return XRB_EINVAL;
            }
        }
    const double R = prm.radius;
    geo.n = (int)n;
    // the kernels' cell order: internal cell p is the caller's cell perm[p]
    geo.perm.resize((size_t)n);
    std::iota(geo.perm.begin(), geo.perm.end(), 0);
    bisect_cells(mesh.xyz, geo.perm.data(), n);
    std::vector<int32_t> inv((size_t)n);
    for (int64_t p = 0; p < n; ++p) inv[(size_t)geo.perm[p]] = (int32_t)p;
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

    for (int64_t p = 0; p < n; ++p) {
        const int64_t i = geo.perm[p];   // the caller's number of internal cell p
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
            const size_t k = 6 * (size_t)p + s;     // cell-major: the 6 slots of a cell are contiguous
            if (s >= d) {                      // pentagon padding: self, zero weights
                geo.nbr[k] = (int32_t)p;
                continue;
            }
            const int32_t j = mesh.nbr[6 * i + s];
            if (j == i) {
                err = "mesh: neighbour index out of range";
                return XRB_EINVAL;
            }
            geo.nbr[k] = inv[(size_t)j];
            const V3 xj = X(j);
            const double le = R * angle(CRN(i, (s + d - 1) % d), CRN(i, s));
            const double de = R * angle(xi, xj);
            const double chord = len(sub(xj, xi));
            geo.alpha[k] = le / (2.0 * area * chord);
            geo.cl[k] = le / (de * area);
        }
        double *ce = &geo.cen[4 * (size_t)p];
        ce[0] = xi.x; ce[1] = xi.y; ce[2] = xi.z;
        ce[3] = 1.0 / area;
        geo.area[p] = area;
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
    // the product's weight series hold for half-chords y with y^2 <= kShortY2MaxHost
    double y2max = 0.0;
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < 6; ++s) {
            const int j = geo.nbr[6 * (size_t)i + s];
            double y2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double dx = geo.cen[4 * (size_t)j + c] - geo.cen[4 * (size_t)i + c];
                y2 += 0.25 * dx * dx;
            }
            if (y2 > kShortY2MaxHost) return;   // tables stay empty: the product keeps its gathers
            y2max = std::max(y2max, y2);
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
    geo.short_terms = y2max <= kShort4Y2MaxHost ? 4 : 5;
}

}  // namespace xrb
