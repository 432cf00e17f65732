// Host-side cavity geometries and cut-fraction arrays (setup step).
#pragma once

#include <functional>
#include <memory>
#include <vector>

#include "dm_internal.h"

namespace dm {

// computed fractions below this are rounding noise of tangencies and set to 0
constexpr double kZeroFraction = 1e-12;

// A cavity interior Omega (open set).  Coordinates are physical; the grid
// origin is 0.  Every method answers for the closed box / segment / face given.
struct Body {
    virtual ~Body() {}
    // 1: the closed box lies in Omega; 0: it does not meet Omega; -1: cut
    virtual int classify(const double *lo, const double *hi) const = 0;
    // length of {p + t e_axis : t in [lo, hi]} inside Omega
    virtual double edge_len(int axis, double lo, double hi, const double *p) const = 0;
    // area inside Omega of the axis-normal face at coordinate c over
    // [lo2[0],hi2[0]] x [lo2[1],hi2[1]] (other two axes in increasing order)
    virtual double face_area(int axis, double c, const double *lo2, const double *hi2) const = 0;
    // volume inside Omega of the box [lo, hi]
    virtual double cell_vol(const double *lo, const double *hi) const = 0;
};

std::unique_ptr<Body> make_body(const dm_geometry &g);
double disk_rect_area(double rho, double x0, double x1, double y0, double y1);
// integral of f over [a, b], split at `cuts` (kinks of f), each piece by
// Gauss--Legendre after a map that flattens endpoint (x - a)^{1/2..3/2} terms
double integrate_pieces(const std::function<double(double)> &f, double a, double b,
                        std::vector<double> cuts);
void compute_fractions(const Body &body, const Grid &g, const int bc_lo[3],
                       std::vector<double> &out);
// fractions of {phi < 0} for phi sampled on the nodes of the grid refined s
// times per cell, interpolated linearly on the Kuhn tetrahedra of the
// refined lattice (geometry_levelset.cpp)
void compute_levelset_fractions(const Grid &g, const double *phi, int s, const int bc_lo[3],
                                std::vector<double> &out);
void enforce_fraction_consistency(const Grid &g, std::vector<double> &fr);
void neglect_faces(const Grid &g, double a_min, std::vector<double> &fr);
void mirror_fraction_ghosts(const Grid &g, std::vector<double> &fr);
void coarsen_fractions(const Grid &gf, const std::vector<double> &ff, const Grid &gc,
                       std::vector<double> &fc);

}  // namespace dm
