// Elliptic-cell body of revolution (multi-cell accelerator cavity profile).
//
// The cavity is {z0 < z < z_end, |(x, y) - axis| < r(z)}: a beam tube of
// radius r_iris and length `tube`, n_cells cells whose radius rises along an
// elliptic arc from r_iris at the cell ends to r_equator at the cell middle,
// and a second tube; conducting end plates close it.  Fractions (Sec. 2 and
// Sec. 5.1 definitions) are closed forms where the cut is a circle or a line
// (z-faces, z-edges, x/y-edges) and 1-D integrals over z otherwise, split at
// the irises and wherever r(z) passes a face corner or side distance.
#include <algorithm>
#include <cmath>
#include <vector>

#include "geometry.h"

namespace dm {

namespace {

struct EllipticBor final : Body {
    double ax, ay, z0, zend, req, rir, L, tube;
    int nc;

    explicit EllipticBor(const dm_geometry &g)
        : ax(g.axis_xy[0]), ay(g.axis_xy[1]), z0(g.z_start), req(g.r_equator), rir(g.r_iris),
          L(g.cell_length), tube(g.tube_length), nc(g.n_cells) {
        zend = z0 + 2.0 * tube + nc * L;
    }
    double centre(int m) const { return z0 + tube + (m + 0.5) * L; }

    double radius(double z) const {
        if (!(z > z0 && z < zend)) return 0.0;
        const double c0 = z0 + tube;
        const int m = (int)std::floor((z - c0) / L);
        if (m >= 0 && m < nc) {
            const double t = (z - centre(m)) / (0.5 * L);
            if (std::fabs(t) < 1.0) return rir + (req - rir) * std::sqrt(1.0 - t * t);
        }
        return rir;
    }
    // limits at the end plates count as the tube radius (for bounds only)
    double rlim(double z) const { return (z <= z0 || z >= zend) ? rir : radius(z); }

    // intervals of z where r(z) > R
    void above(double R, std::vector<std::pair<double, double>> &out) const {
        out.clear();
        if (R < rir) {
            out.emplace_back(z0, zend);
            return;
        }
        if (R >= req) return;
        const double t = (R - rir) / (req - rir);
        const double half = 0.5 * L * std::sqrt(1.0 - t * t);
        for (int m = 0; m < nc; ++m) out.emplace_back(centre(m) - half, centre(m) + half);
    }
    void add_crossings(double R, double lo, double hi, std::vector<double> &pts) const {
        std::vector<std::pair<double, double>> iv;
        above(R, iv);
        for (auto &p : iv) {
            if (p.first > lo && p.first < hi) pts.push_back(p.first);
            if (p.second > lo && p.second < hi) pts.push_back(p.second);
        }
    }
    void add_junctions(double lo, double hi, std::vector<double> &pts) const {
        const double c0 = z0 + tube;
        for (int m = 0; m <= nc; ++m) {
            const double z = c0 + m * L;
            if (z > lo && z < hi) pts.push_back(z);
        }
        if (z0 > lo && z0 < hi) pts.push_back(z0);
        if (zend > lo && zend < hi) pts.push_back(zend);
    }

    int classify(const double *lo, const double *hi) const override {
        if (hi[2] <= z0 || lo[2] >= zend) return 0;
        const double dx0 = lo[0] - ax, dx1 = hi[0] - ax, dy0 = lo[1] - ay, dy1 = hi[1] - ay;
        const double far = std::sqrt(std::max(dx0 * dx0, dx1 * dx1) + std::max(dy0 * dy0, dy1 * dy1));
        const double nx = (dx0 <= 0.0 && dx1 >= 0.0) ? 0.0 : std::min(std::fabs(dx0), std::fabs(dx1));
        const double ny = (dy0 <= 0.0 && dy1 >= 0.0) ? 0.0 : std::min(std::fabs(dy0), std::fabs(dy1));
        const double near = std::sqrt(nx * nx + ny * ny);
        const double a = std::max(lo[2], z0), b = std::min(hi[2], zend);
        std::vector<double> zs = {a, b};
        add_junctions(a, b, zs);
        double rmin = INFINITY, rmax = 0.0;
        for (double z : zs) {
            rmin = std::min(rmin, rlim(z));
            rmax = std::max(rmax, rlim(z));
        }
        for (int m = 0; m < nc; ++m)
            if (centre(m) > a && centre(m) < b) rmax = std::max(rmax, req);
        if (near >= rmax) return 0;
        if (far < rmin && lo[2] > z0 && hi[2] < zend) return 1;
        return -1;
    }

    double edge_len(int axis, double lo, double hi, const double *p) const override {
        if (axis == 2) {
            const double rho = std::hypot(p[0] - ax, p[1] - ay);
            std::vector<std::pair<double, double>> iv;
            above(rho, iv);
            double s = 0.0;
            for (auto &q : iv) s += std::max(0.0, std::min(hi, q.second) - std::max(lo, q.first));
            return s;
        }
        const double r = radius(p[2]);
        const double other = axis == 0 ? p[1] - ay : p[0] - ax;
        if (r <= std::fabs(other)) return 0.0;
        const double s = std::sqrt(r * r - other * other);
        const double c = axis == 0 ? ax : ay;
        return std::max(0.0, std::min(hi, c + s) - std::max(lo, c - s));
    }

    double face_area(int axis, double c, const double *lo2, const double *hi2) const override {
        if (axis == 2) return disk_rect_area(radius(c), lo2[0] - ax, hi2[0] - ax, lo2[1] - ay, hi2[1] - ay);
        // x-face: (y, z); y-face: (x, z)
        const double d = c - (axis == 0 ? ax : ay);
        const double cen = axis == 0 ? ay : ax;
        const double t0 = lo2[0] - cen, t1 = hi2[0] - cen, zlo = lo2[1], zhi = hi2[1];
        auto chord = [&](double z) {
            const double r = radius(z);
            if (r <= std::fabs(d)) return 0.0;
            const double s = std::sqrt(r * r - d * d);
            return std::max(0.0, std::min(t1, s) - std::max(t0, -s));
        };
        std::vector<double> cuts;
        add_junctions(zlo, zhi, cuts);
        for (double R : {std::fabs(d), std::hypot(d, t0), std::hypot(d, t1)}) add_crossings(R, zlo, zhi, cuts);
        return integrate_pieces(chord, zlo, zhi, cuts);
    }

    double cell_vol(const double *lo, const double *hi) const override {
        const double x0 = lo[0] - ax, x1 = hi[0] - ax, y0 = lo[1] - ay, y1 = hi[1] - ay;
        auto area = [&](double z) { return disk_rect_area(radius(z), x0, x1, y0, y1); };
        std::vector<double> cuts;
        add_junctions(lo[2], hi[2], cuts);
        const double ds[8] = {std::fabs(x0), std::fabs(x1), std::fabs(y0), std::fabs(y1),
                              std::hypot(x0, y0), std::hypot(x0, y1), std::hypot(x1, y0), std::hypot(x1, y1)};
        for (double R : ds) add_crossings(R, lo[2], hi[2], cuts);
        return integrate_pieces(area, lo[2], hi[2], cuts);
    }
};

}  // namespace

std::unique_ptr<Body> make_elliptic_bor(const dm_geometry &g) {
    if (!(g.n_cells >= 1 && g.r_iris > 0.0 && g.r_equator > g.r_iris && g.cell_length > 0.0 &&
          g.tube_length >= 0.0))
        return nullptr;
    return std::unique_ptr<Body>(new EllipticBor(g));
}

}  // namespace dm
