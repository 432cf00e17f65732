// Cut fractions of a general cavity given by a level set (Sec. 6.1: cut-cell
// volumes from tetrahedral subvolumes that conform to the embedded surface).
//
// The caller samples phi (< 0 in the cavity, >= 0 in the conductor) on the
// nodes of the grid refined s times per cell.  The cavity is taken to be
// {phi_lin < 0} for the piecewise-linear interpolant of phi on the Kuhn
// (Freudenthal) triangulation of the refined lattice: every refined cube is
// cut into the 6 tetrahedra that share its main diagonal, so every cube
// face is split into 2 triangles along the diagonal through its lowest and
// highest corner, the same for the two cubes that share it.  The surface is
// then a polyhedron whose facets are planar inside each tetrahedron, and
// the fractions are exact for it: a cell's volume is the sum over its
// tetrahedra of the part where phi_lin < 0 (a tetrahedron, its complement,
// or a triangular prism cut by the facet), a face's area the same over its
// triangles, an edge's length over its refined segments.  Cells, faces and
// edges of one grid therefore measure one body consistently, and the
// fractions converge to those of the smooth surface as the refinement grows
// (at second order in h / s for a smooth phi).
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "geometry.h"

namespace dm {

namespace {

// cut parameter along a -> b of the zero of the linear interpolant, a < 0 <= b
inline double cut_t(double a, double b) { return a / (a - b); }

// part of [0, 1] where the linear interpolant of (p0, p1) is negative
double seg_neg(double p0, double p1) {
    const bool n0 = p0 < 0.0, n1 = p1 < 0.0;
    if (n0 && n1) return 1.0;
    if (!n0 && !n1) return 0.0;
    return n0 ? cut_t(p0, p1) : cut_t(p1, p0);
}

// part of a triangle's area where the linear interpolant of its vertex
// values is negative: a corner triangle (one negative vertex) or the
// complement of one (one non-negative vertex)
double tri_neg(const double p[3]) {
    int neg = 0;
    for (int q = 0; q < 3; ++q) neg += p[q] < 0.0;
    if (neg == 0) return 0.0;
    if (neg == 3) return 1.0;
    const bool one = neg == 1;
    int s = 0;   // the odd vertex out
    for (int q = 0; q < 3; ++q)
        if ((p[q] < 0.0) == one) s = q;
    // the corner triangle at the odd vertex: its legs along the two edges are
    // the parameters of the zero measured from that vertex, a / (a - x)
    const double a = p[s], b = p[(s + 1) % 3], c = p[(s + 2) % 3];
    const double corner = (a / (a - b)) * (a / (a - c));
    return one ? corner : 1.0 - corner;
}

inline double det3(const double u[3], const double v[3], const double w[3]) {
    return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) + u[2] * (v[0] * w[1] - v[1] * w[0]);
}

// volume of the tetrahedron (a, b, c, d)
inline double tet_vol(const double *a, const double *b, const double *c, const double *d) {
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double v[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double w[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    return std::fabs(det3(u, v, w)) / 6.0;
}

// part of a tetrahedron's volume (vertices X, values p) where the linear
// interpolant is negative
double tet_neg(const double p[4], const double X[4][3]) {
    int neg = 0;
    for (int q = 0; q < 4; ++q) neg += p[q] < 0.0;
    if (neg == 0) return 0.0;
    if (neg == 4) return 1.0;
    if (neg == 1 || neg == 3) {
        // a corner tetrahedron at the odd vertex out: the product of the
        // zero's parameters along its three edges, measured from that vertex
        const bool one = neg == 1;
        int s = 0;
        for (int q = 0; q < 4; ++q)
            if ((p[q] < 0.0) == one) s = q;
        double corner = 1.0;
        for (int q = 0; q < 4; ++q)
            if (q != s) corner *= p[s] / (p[s] - p[q]);
        return one ? corner : 1.0 - corner;
    }
    // two negative vertices a, b and two others c, d: the negative part is the
    // prism with triangles (a, P_ac, P_ad) and (b, P_bc, P_bd), cut into the
    // three tetrahedra (A B C D), (B C D E), (C D E F) of prism ABC-DEF
    int ng[2], ps[2], in = 0, ip = 0;
    for (int q = 0; q < 4; ++q) (p[q] < 0.0 ? ng[in++] : ps[ip++]) = q;
    auto cut_point = [&](int from, int to, double out[3]) {
        const double t = cut_t(p[from], p[to]);
        for (int c = 0; c < 3; ++c) out[c] = X[from][c] + t * (X[to][c] - X[from][c]);
    };
    double A[3], B[3], C[3], D[3], E[3], F[3];
    for (int c = 0; c < 3; ++c) {
        A[c] = X[ng[0]][c];
        D[c] = X[ng[1]][c];
    }
    cut_point(ng[0], ps[0], B);
    cut_point(ng[0], ps[1], C);
    cut_point(ng[1], ps[0], E);
    cut_point(ng[1], ps[1], F);
    const double vol = tet_vol(A, B, C, D) + tet_vol(B, C, D, E) + tet_vol(C, D, E, F);
    return vol / tet_vol(X[0], X[1], X[2], X[3]);
}

// part of the refined unit cube (corner values c[dx + 2 dy + 4 dz]) where the
// interpolant on its 6 Kuhn tetrahedra is negative
double cube_neg(const double c[8]) {
    bool any_neg = false, any_pos = false;
    for (int q = 0; q < 8; ++q) (c[q] < 0.0 ? any_neg : any_pos) = true;
    if (!any_neg) return 0.0;
    if (!any_pos) return 1.0;
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    double sum = 0.0;
    for (int t = 0; t < 6; ++t) {
        int v[4] = {0, 0, 0, 7};
        v[1] = 1 << perm[t][0];
        v[2] = v[1] | (1 << perm[t][1]);
        double X[4][3], p[4];
        for (int q = 0; q < 4; ++q) {
            for (int a = 0; a < 3; ++a) X[q][a] = (v[q] >> a) & 1;
            p[q] = c[v[q]];
        }
        sum += tet_neg(p, X);
    }
    return sum / 6.0;
}

}  // namespace

void compute_levelset_fractions(const Grid &g, const double *phi, int s, const int bc_lo[3],
                                std::vector<double> &out) {
    const int64_t P = g.P;
    out.assign(7 * P, 0.0);
    const int n[3] = {g.nx, g.ny, g.nz};
    const int64_t NX = (int64_t)s * g.nx + 1, NY = (int64_t)s * g.ny + 1;
    auto node = [&](int64_t I, int64_t J, int64_t K) { return phi[I + NX * (J + NY * K)]; };
    auto clean = [](double v) { return v >= kZeroFraction ? v : 0.0; };
    // as for the analytic bodies: a face/edge in a low-side wall is active
    // only on a PMC plane; high-side walls are perfect electric conductors
    auto in_wall = [&](int a, int idx) { return (idx == 0 && bc_lo[a] != DM_BC_PMC) || idx == n[a]; };
    const double inv_s = 1.0 / s, inv_s2 = inv_s * inv_s, inv_s3 = inv_s2 * inv_s;
    auto work = [&](int k0, int k1) {
        for (int k = k0; k < k1; ++k)
            for (int j = 0; j <= g.ny; ++j)
                for (int i = 0; i <= g.nx; ++i) {
                    const int idx[3] = {i, j, k};
                    const int64_t p = pidx(g, i, j, k);
                    const int64_t base[3] = {(int64_t)s * i, (int64_t)s * j, (int64_t)s * k};
                    for (int a = 0; a < 3; ++a) {
                        const int b = a == 0 ? 1 : 0, d = a == 2 ? 1 : 2;
                        // face normal to a: sub-squares over axes b < d, each
                        // split along the diagonal (0,0)-(1,1)
                        if (idx[b] < n[b] && idx[d] < n[d] && idx[a] <= n[a] && !in_wall(a, idx[a])) {
                            double sum = 0.0;
                            for (int u = 0; u < s; ++u)
                                for (int w = 0; w < s; ++w) {
                                    double cq[4];   // (u,w) (u+1,w) (u,w+1) (u+1,w+1)
                                    for (int q = 0; q < 4; ++q) {
                                        int64_t I[3] = {base[0], base[1], base[2]};
                                        I[b] += u + (q & 1);
                                        I[d] += w + (q >> 1);
                                        cq[q] = node(I[0], I[1], I[2]);
                                    }
                                    const double t1[3] = {cq[0], cq[1], cq[3]}, t2[3] = {cq[0], cq[2], cq[3]};
                                    sum += 0.5 * (tri_neg(t1) + tri_neg(t2));
                                }
                            out[a * P + p] = clean(sum * inv_s2);
                        }
                        // edge along a
                        if (idx[a] < n[a] && idx[b] <= n[b] && idx[d] <= n[d] && !in_wall(b, idx[b]) &&
                            !in_wall(d, idx[d])) {
                            double sum = 0.0;
                            for (int u = 0; u < s; ++u) {
                                int64_t I0[3] = {base[0], base[1], base[2]}, I1[3] = {base[0], base[1], base[2]};
                                I0[a] += u;
                                I1[a] += u + 1;
                                sum += seg_neg(node(I0[0], I0[1], I0[2]), node(I1[0], I1[1], I1[2]));
                            }
                            out[(3 + a) * P + p] = clean(sum * inv_s);
                        }
                    }
                    if (i < g.nx && j < g.ny && k < g.nz) {
                        double sum = 0.0;
                        for (int cz = 0; cz < s; ++cz)
                            for (int cy = 0; cy < s; ++cy)
                                for (int cx = 0; cx < s; ++cx) {
                                    double c[8];
                                    for (int q = 0; q < 8; ++q)
                                        c[q] = node(base[0] + cx + (q & 1), base[1] + cy + ((q >> 1) & 1),
                                                    base[2] + cz + (q >> 2));
                                    sum += cube_neg(c);
                                }
                        out[6 * P + p] = clean(sum * inv_s3);
                    }
                }
    };
    const int nk = g.nz + 1;
    int nthreads = (int)std::thread::hardware_concurrency();
    nthreads = std::max(1, std::min({nthreads, 32, nk}));
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
        const int k0 = (int)((int64_t)nk * t / nthreads), k1 = (int)((int64_t)nk * (t + 1) / nthreads);
        th.emplace_back(work, k0, k1);
    }
    for (auto &t : th) t.join();
}

}  // namespace dm
