// Cut-cell fractions of the Dey--Mittra method on the host (setup step).
//
// Sec. 2 (after eq. farInt): a cut face / edge keeps the portion of its area /
// length outside the conductor, divided by h^2 / h.  Sec. 5.1 (after
// eq. divBInt): a cut cell keeps its volume outside the conductor over h^3.
//
// Formulation used here:
//  * area of a rectangle inside a disk = difference of two "strips", each the
//    integral over x of the part of the chord (-s(x), s(x)) below a line
//    y = Y, integrated in closed form with the antiderivative of
//    sqrt(rho^2 - x^2);
//  * a volume = integral of the cross-section area along x, by 48-point
//    Gauss--Legendre on each interval between the kinks of the section area,
//    after the map x = a + (b - a)(3t^2 - 2t^3) that flattens the
//    (x - kink)^{3/2} behaviour at both interval ends;
//  * bodies of revolution: the same with the section radius given by the
//    radius profile r(z).
// Fractions below kZeroFraction are rounding noise of tangencies and set 0.
#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>
#include <vector>

#include "dm_internal.h"
#include "geometry.h"

namespace dm {

namespace {

// Gauss--Legendre nodes/weights on [0,1], computed once by Newton iteration
struct GaussLegendre {
    std::vector<double> x, w;
    explicit GaussLegendre(int n) : x(n), w(n) {
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                const double dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            x[i] = 0.5 * (1.0 - z);
            w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 2/((1-z^2)dp^2) / 2
        }
    }
};

const GaussLegendre &gl48() {
    static const GaussLegendre g(48);
    return g;
}

// integral of f over [a,b] with kink-flattening map on both ends
double integrate_smooth(const std::function<double(double)> &f, double a, double b) {
    if (!(b > a)) return 0.0;
    const GaussLegendre &g = gl48();
    const double L = b - a;
    double s = 0.0;
    for (size_t i = 0; i < g.x.size(); ++i) {
        const double t = g.x[i];
        const double phi = t * t * (3.0 - 2.0 * t);
        const double dphi = 6.0 * t * (1.0 - t);
        s += g.w[i] * dphi * f(a + L * phi);
    }
    return s * L;
}

}  // namespace

double integrate_pieces(const std::function<double(double)> &f, double a, double b,
                        std::vector<double> cuts) {
    cuts.push_back(a);
    cuts.push_back(b);
    std::sort(cuts.begin(), cuts.end());
    double s = 0.0;
    double prev = a;
    for (double c : cuts) {
        if (c <= prev || c > b) continue;
        s += integrate_smooth(f, prev, c);
        prev = c;
    }
    return s;
}

namespace {

// antiderivative of sqrt(rho^2 - t^2), t clamped to [-rho, rho]
inline double arc_prim(double t, double rho) {
    t = std::min(std::max(t, -rho), rho);
    return 0.5 * (t * std::sqrt(std::max(rho * rho - t * t, 0.0)) + rho * rho * std::asin(t / rho));
}

// integral over x in [x0,x1] of |(-s(x), s(x)) intersect (-inf, Y)|
double strip_below(double x0, double x1, double Y, double rho) {
    x0 = std::max(x0, -rho);
    x1 = std::min(x1, rho);
    if (x1 <= x0) return 0.0;
    const double full = 2.0 * (arc_prim(x1, rho) - arc_prim(x0, rho));
    if (Y >= rho) return full;
    if (Y <= -rho) return 0.0;
    const double w = std::sqrt(rho * rho - Y * Y);
    const double a = std::max(x0, -w), b = std::min(x1, w);
    double mid = 0.0, len = 0.0;
    if (b > a) {
        mid = arc_prim(b, rho) - arc_prim(a, rho);
        len = b - a;
    }
    return Y >= 0.0 ? full - (mid - Y * len) : mid + Y * len;
}

}  // namespace

double disk_rect_area(double rho, double x0, double x1, double y0, double y1) {
    if (rho <= 0.0 || x1 <= x0 || y1 <= y0) return 0.0;
    const double v = strip_below(x0, x1, y1, rho) - strip_below(x0, x1, y0, rho);
    return v > 0.0 ? v : 0.0;
}

// ---------------------------------------------------------------------------
// Ellipsoid: computed in u = (x - c) / s where the cavity is the unit ball
// ---------------------------------------------------------------------------
struct Ellipsoid final : Body {
    double c[3], s[3];
    Ellipsoid(const double *cen, const double *semi) {
        for (int a = 0; a < 3; ++a) {
            c[a] = cen[a];
            s[a] = semi[a];
        }
    }
    double u(int a, double x) const { return (x - c[a]) / s[a]; }

    int classify(const double *lo, const double *hi) const override {
        double far = 0.0, near = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double l = u(a, lo[a]), h = u(a, hi[a]);
            far += std::max(l * l, h * h);
            if (l > 0.0) near += l * l;
            else if (h < 0.0) near += h * h;
        }
        if (far < 1.0) return 1;
        if (near >= 1.0) return 0;
        return -1;
    }
    double edge_len(int axis, double lo, double hi, const double *p) const override {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a)
            if (a != axis) d2 += u(a, p[a]) * u(a, p[a]);
        if (d2 >= 1.0) return 0.0;
        const double half = std::sqrt(1.0 - d2) * s[axis];
        return std::max(0.0, std::min(hi, c[axis] + half) - std::max(lo, c[axis] - half));
    }
    double section_u(double uc, double ulo0, double uhi0, double ulo1, double uhi1) const {
        const double r2 = 1.0 - uc * uc;
        if (r2 <= 0.0) return 0.0;
        return disk_rect_area(std::sqrt(r2), ulo0, uhi0, ulo1, uhi1);
    }
    double face_area(int axis, double cc, const double *lo2, const double *hi2) const override {
        const int b = axis == 0 ? 1 : 0, d = axis == 2 ? 1 : 2;
        return section_u(u(axis, cc), u(b, lo2[0]), u(b, hi2[0]), u(d, lo2[1]), u(d, hi2[1])) *
               s[b] * s[d];
    }
    double cell_vol(const double *lo, const double *hi) const override {
        double ul[3], uh[3];
        for (int a = 0; a < 3; ++a) {
            ul[a] = u(a, lo[a]);
            uh[a] = u(a, hi[a]);
        }
        std::vector<double> d = {0.0, std::fabs(ul[1]), std::fabs(uh[1]), std::fabs(ul[2]),
                                 std::fabs(uh[2])};
        for (double y : {ul[1], uh[1]})
            for (double z : {ul[2], uh[2]}) d.push_back(std::sqrt(y * y + z * z));
        std::vector<double> cuts;
        for (double dd : d)
            if (dd < 1.0) {
                const double r = std::sqrt(1.0 - dd * dd);
                cuts.push_back(-r);
                cuts.push_back(r);
            }
        auto f = [&](double ux) { return section_u(ux, ul[1], uh[1], ul[2], uh[2]); };
        return integrate_pieces(f, ul[0], uh[0], cuts) * s[0] * s[1] * s[2];
    }
};

// ---------------------------------------------------------------------------
// Box cavity: the whole domain box (only the walls conduct)
// ---------------------------------------------------------------------------
struct WholeBox final : Body {
    int classify(const double *, const double *) const override { return 1; }
    double edge_len(int, double lo, double hi, const double *) const override { return hi - lo; }
    double face_area(int, double, const double *lo2, const double *hi2) const override {
        return (hi2[0] - lo2[0]) * (hi2[1] - lo2[1]);
    }
    double cell_vol(const double *lo, const double *hi) const override {
        return (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    }
};

std::unique_ptr<Body> make_elliptic_bor(const dm_geometry &g);  // geometry_bor.cpp

std::unique_ptr<Body> make_body(const dm_geometry &g) {
    switch (g.kind) {
        case DM_GEOM_BOX: return std::unique_ptr<Body>(new WholeBox());
        case DM_GEOM_ELLIPSOID: return std::unique_ptr<Body>(new Ellipsoid(g.center, g.semi_axes));
        case DM_GEOM_ELLIPTIC_BOR: return make_elliptic_bor(g);
        default: return nullptr;
    }
}

// ---------------------------------------------------------------------------
// fraction arrays of the finest grid (7 padded blocks: ax ay az lx ly lz v)
// ---------------------------------------------------------------------------
void compute_fractions(const Body &body, const Grid &g, const int bc_lo[3],
                       std::vector<double> &out) {
    const int64_t P = g.P;
    out.assign(7 * P, 0.0);
    const int n[3] = {g.nx, g.ny, g.nz};
    const double h = g.h;
    auto clean = [](double v) { return v >= kZeroFraction ? v : 0.0; };
    // a face/edge in a low-side wall is active only on a PMC symmetry plane;
    // high-side walls are always perfect electric conductors
    auto in_wall = [&](int a, int idx) {
        return (idx == 0 && bc_lo[a] != DM_BC_PMC) || idx == n[a];
    };
    auto work = [&](int k0, int k1) {
        for (int k = k0; k < k1; ++k)
            for (int j = 0; j <= g.ny; ++j)
                for (int i = 0; i <= g.nx; ++i) {
                    const int idx[3] = {i, j, k};
                    const int64_t p = pidx(g, i, j, k);
                    // faces: normal axis a, spans the other two within the grid
                    for (int a = 0; a < 3; ++a) {
                        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
                        if (idx[b] >= n[b] || idx[d] >= n[d] || idx[a] > n[a]) continue;
                        if (in_wall(a, idx[a])) continue;
                        double lo[3] = {i * h, j * h, k * h}, hi[3] = {i * h, j * h, k * h};
                        hi[b] += h;
                        hi[d] += h;
                        const int cls = body.classify(lo, hi);
                        double v = 0.0;
                        if (cls == 1) v = 1.0;
                        else if (cls < 0) {
                            const double lo2[2] = {lo[b], lo[d]}, hi2[2] = {hi[b], hi[d]};
                            v = clean(body.face_area(a, idx[a] * h, lo2, hi2) / (h * h));
                        }
                        out[a * P + p] = v;
                    }
                    // edges along axis a, lying at node coordinates of the others
                    for (int a = 0; a < 3; ++a) {
                        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
                        if (idx[a] >= n[a] || idx[b] > n[b] || idx[d] > n[d]) continue;
                        if (in_wall(b, idx[b]) || in_wall(d, idx[d])) continue;
                        const double pt[3] = {i * h, j * h, k * h};
                        double lo[3] = {pt[0], pt[1], pt[2]}, hi[3] = {pt[0], pt[1], pt[2]};
                        hi[a] += h;
                        const int cls = body.classify(lo, hi);
                        double v = 0.0;
                        if (cls == 1) v = 1.0;
                        else if (cls < 0) v = clean(body.edge_len(a, pt[a], pt[a] + h, pt) / h);
                        out[(3 + a) * P + p] = v;
                    }
                    // cell
                    if (i < g.nx && j < g.ny && k < g.nz) {
                        const double lo[3] = {i * h, j * h, k * h};
                        const double hi[3] = {lo[0] + h, lo[1] + h, lo[2] + h};
                        const int cls = body.classify(lo, hi);
                        double v = 0.0;
                        if (cls == 1) v = 1.0;
                        else if (cls < 0) v = clean(body.cell_vol(lo, hi) / (h * h * h));
                        out[6 * P + p] = v;
                    }
                }
    };
    const int nk = g.nz + 1;
    int nthreads = (int)std::thread::hardware_concurrency();
    nthreads = std::max(1, std::min(nthreads, 32));
    nthreads = std::min(nthreads, nk);
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
        const int k0 = (int)((int64_t)nk * t / nthreads), k1 = (int)((int64_t)nk * (t + 1) / nthreads);
        th.emplace_back(work, k0, k1);
    }
    for (auto &t : th) t.join();
}

// PMC ghost layer of the fraction blocks: the mirror image of the cavity
// across each low-side PMC plane (planes in the order x, y, z so corners
// get both mirrors).  Across the plane normal to a, a node-centred quantity
// (face normal to a, edge across a) at -1 mirrors +1; a cell-centred one
// (other faces, edge along a, cell) at -1 mirrors 0.
void mirror_fraction_ghosts(const Grid &g, std::vector<double> &fr) {
    if (!g.pmc) return;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t stride[3] = {1, g.sy, g.sz};
    for (int a = 0; a < 3; ++a) {
        if (!((g.pmc >> a) & 1)) continue;
        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
        for (int u = -1; u <= n[b]; ++u)
            for (int v = -1; v <= n[d]; ++v) {
                int idx[3];
                idx[a] = -1;
                idx[b] = u;
                idx[d] = v;
                const int64_t pg = pidx(g, idx[0], idx[1], idx[2]);
                for (int blk = 0; blk < 7; ++blk) {
                    // node-centred along a: face blk==a, edges 3+e with e != a
                    const bool node = (blk < 3 && blk == a) || (blk >= 3 && blk < 6 && blk - 3 != a);
                    fr[blk * g.P + pg] = fr[blk * g.P + pg + (node ? 2 : 1) * stride[a]];
                }
            }
    }
}

// Consistency of thresholded fractions.  Exact fractions of an open cavity
// have area on both sides of a face with area and on all four faces around an
// edge with length; rounding tangencies to 0 can break both.  A face next to
// a cell without volume (a sliver whose volume fell below kZeroFraction while
// its area, of lower order in the thickness, did not) would keep a flux with
// no divergence penalty, a near-null mode of M: it is dropped.  Then every
// edge of a face without area is dropped too (as face neglect does), so that
// the gradients D^T psi on the active faces stay curl-free.  Only cells and
// faces inside the grid are looked at; the ghost images across a PMC plane
// equal their originals.
void enforce_fraction_consistency(const Grid &g, std::vector<double> &fr) {
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t stride[3] = {1, g.sy, g.sz};
    const double *v = &fr[6 * P];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n[2] + (a == 2); ++k)
            for (int j = 0; j < n[1] + (a == 1); ++j)
                for (int i = 0; i < n[0] + (a == 0); ++i) {
                    const int64_t p = pidx(g, i, j, k);
                    if (fr[a * P + p] == 0.0) continue;
                    const int idx = a == 0 ? i : a == 1 ? j : k;
                    const bool lo_empty = idx > 0 && v[p - stride[a]] == 0.0;
                    const bool hi_empty = idx < n[a] && v[p] == 0.0;
                    if (lo_empty || hi_empty) fr[a * P + p] = 0.0;
                }
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n[2] + (a == 2); ++k)
            for (int j = 0; j < n[1] + (a == 1); ++j)
                for (int i = 0; i < n[0] + (a == 0); ++i) {
                    const int64_t p = pidx(g, i, j, k);
                    if (fr[a * P + p] != 0.0) continue;
                    if (a == 0) {          // x-face: e_y(p), e_y(p+dz), e_z(p), e_z(p+dy)
                        fr[4 * P + p] = fr[4 * P + p + dz] = 0.0;
                        fr[5 * P + p] = fr[5 * P + p + dy] = 0.0;
                    } else if (a == 1) {   // y-face: e_x(p), e_x(p+dz), e_z(p), e_z(p+1)
                        fr[3 * P + p] = fr[3 * P + p + dz] = 0.0;
                        fr[5 * P + p] = fr[5 * P + p + 1] = 0.0;
                    } else {               // z-face: e_x(p), e_x(p+dy), e_y(p), e_y(p+1)
                        fr[3 * P + p] = fr[3 * P + p + dy] = 0.0;
                        fr[4 * P + p] = fr[4 * P + p + 1] = 0.0;
                    }
                }
}

// Face neglect (Sec. 3): faces with 0 < a < a_min lose their b (a := 0) and
// every edge around such a face its e (l := 0).
void neglect_faces(const Grid &g, double a_min, std::vector<double> &fr) {
    if (!(a_min > 0.0)) return;
    const int64_t P = g.P, dy = g.sy, dz = g.sz;
    std::vector<int64_t> drop[3];
    for (int a = 0; a < 3; ++a)
        for (int64_t p = 0; p < P; ++p) {
            const double v = fr[a * P + p];
            if (v > 0.0 && v < a_min) drop[a].push_back(p);
        }
    for (int a = 0; a < 3; ++a)
        for (int64_t p : drop[a]) {
            fr[a * P + p] = 0.0;
            if (a == 0) {          // x-face: edges e_y(p), e_y(p+dz), e_z(p), e_z(p+dy)
                fr[4 * P + p] = fr[4 * P + p + dz] = 0.0;
                fr[5 * P + p] = fr[5 * P + p + dy] = 0.0;
            } else if (a == 1) {   // y-face: e_x(p), e_x(p+dz), e_z(p), e_z(p+1)
                fr[3 * P + p] = fr[3 * P + p + dz] = 0.0;
                fr[5 * P + p] = fr[5 * P + p + 1] = 0.0;
            } else {               // z-face: e_x(p), e_x(p+dy), e_y(p), e_y(p+1)
                fr[3 * P + p] = fr[3 * P + p + dy] = 0.0;
                fr[4 * P + p] = fr[4 * P + p + 1] = 0.0;
            }
        }
    // a cell left without any open face holds no field: its volume goes too
    // (else its scalar unknown is an island of the projection's D A D^T)
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const int64_t p = pidx(g, i, j, k);
                if (!(fr[6 * P + p] > 0.0)) continue;
                const bool open = fr[p] > 0.0 || fr[p + 1] > 0.0 || fr[P + p] > 0.0 || fr[P + p + dy] > 0.0 ||
                                  fr[2 * P + p] > 0.0 || fr[2 * P + p + dz] > 0.0;
                if (!open) fr[6 * P + p] = 0.0;
            }
}

// Coarse fractions: a coarse face is the union of its 4 sub-faces, a coarse
// edge of its 2 sub-edges and a coarse cell of its 8 sub-cells.
void coarsen_fractions(const Grid &gf, const std::vector<double> &ff, const Grid &gc,
                       std::vector<double> &fc) {
    const int64_t Pf = gf.P, Pc = gc.P, fy = gf.sy, fz = gf.sz;
    fc.assign(7 * Pc, 0.0);
    for (int K = 0; K <= gc.nz; ++K)
        for (int J = 0; J <= gc.ny; ++J)
            for (int I = 0; I <= gc.nx; ++I) {
                const int64_t pc = pidx(gc, I, J, K);
                const int i = 2 * I, j = 2 * J, k = 2 * K;
                const bool ci = I < gc.nx, cj = J < gc.ny, ck = K < gc.nz;
                const int64_t q = pidx(gf, std::min(i, gf.nx), std::min(j, gf.ny), std::min(k, gf.nz));
                const double *ax = &ff[0], *ay = &ff[Pf], *az = &ff[2 * Pf];
                const double *lx = &ff[3 * Pf], *ly = &ff[4 * Pf], *lz = &ff[5 * Pf];
                const double *v = &ff[6 * Pf];
                if (cj && ck) fc[pc] = 0.25 * (ax[q] + ax[q + fy] + ax[q + fz] + ax[q + fy + fz]);
                if (ci && ck) fc[Pc + pc] = 0.25 * (ay[q] + ay[q + 1] + ay[q + fz] + ay[q + 1 + fz]);
                if (ci && cj) fc[2 * Pc + pc] = 0.25 * (az[q] + az[q + 1] + az[q + fy] + az[q + 1 + fy]);
                if (ci) fc[3 * Pc + pc] = 0.5 * (lx[q] + lx[q + 1]);
                if (cj) fc[4 * Pc + pc] = 0.5 * (ly[q] + ly[q + fy]);
                if (ck) fc[5 * Pc + pc] = 0.5 * (lz[q] + lz[q + fz]);
                if (ci && cj && ck) {
                    double s = 0.0;
                    for (int c = 0; c < 8; ++c) s += v[q + (c & 1) + ((c >> 1) & 1) * fy + (c >> 2) * fz];
                    fc[6 * Pc + pc] = 0.125 * s;
                }
            }
}

}  // namespace dm
