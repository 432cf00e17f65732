"""Oracle: Dey--Mittra cut fractions (TEST INFRASTRUCTURE ONLY).

Definitions followed
--------------------
* Sec. 2 (discussion after eq. farInt): when a face or edge is cut by the
  perfect conductor, its area / length is replaced by the portion lying
  *outside* the conductor; the diagonal matrices of eq. discWaveBDM hold
  these portions divided by the vacuum area h^2 / length h.
* Sec. 5.1 (text after eq. divBInt, eq. divBDM): the cell volume fraction is
  the volume of the cell outside the conductor divided by h^3.

Conventions (this project's readings, stated once):
* cell (i,j,k) is [ih,(i+1)h] x [jh,(j+1)h] x [kh,(k+1)h]; the domain box
  [0,Nx h] x [0,Ny h] x [0,Nz h] is bounded by perfectly conducting walls;
  a face or edge lying in a wall has fraction 0;
* the cavity interior Omega is open and the conductor closed, so a face that
  only touches Omega along a curve has area fraction 0;
* a computed fraction below ZERO_FRACTION (1e-12, far below any fraction
  a resolved boundary produces and above the rounding error of the area and
  volume formulas, ~1e-13) is rounding noise of a tangency and is set to 0;
* two consistency rules then restore what holds for exact fractions of an
  open cavity: a face with area has volume on both sides, and an edge with
  length has area on all four faces around it.  A face next to a cell of
  volume 0 gets a = 0 (a tangency sliver whose volume was rounded away but
  whose area, of lower order in the sliver's thickness, was not: its b would
  carry a flux with no divergence penalty, a near-null mode of M); then every
  edge of a face with a = 0 gets l = 0 (as face neglect does, Sec. 3), so that
  the discrete gradients D^T psi on the active faces stay curl-free.

Array layout: numpy arrays indexed [k, j, i] (x fastest), shapes
    ax (Nz, Ny, Nx+1)   ay (Nz, Ny+1, Nx)   az (Nz+1, Ny, Nx)
    lx (Nz+1, Ny+1, Nx) ly (Nz+1, Ny, Nx+1) lz (Nz, Ny+1, Nx+1)
    v  (Nz, Ny, Nx)

Every routine here is the plain definition: the area of a rectangle inside a
disk is the integral of the chord length (integrated piece by piece with the
antiderivative of sqrt(rho^2 - t^2)), a volume is the integral of the
cross-section area (SciPy adaptive quadrature with the kinks as
breakpoints).  The integrals along the axis are taken piece by piece between
the kinks with the substitution t = end +- s^2 at both ends of every piece:
at an iris two elliptic arcs meet with a vertical tangent (r(z) - r_iris
grows like sqrt|z - z_iris|), and at a pole of an ellipsoid the section
radius grows like the square root of the distance; an adaptive rule applied
to the axis coordinate directly stalled near 1e-11 (iris cells) and 5e-11
(cells touching a pole) in cell units.  Pinned in tests against: measure sums (plane sums of areas
equal the disk area, line sums of lengths equal the chord, the volume sum
equals the ball volume), direct 2-D / 3-D SciPy quadrature of the
indicator on individual faces and cells, the octahedral symmetry of a
node-centred sphere, and the component counts and smallest area fraction
printed in the paper's sphere benchmark (Sec. 6.1, Table tab:invPerf).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import integrate

# ---------------------------------------------------------------------------
# 1-D / 2-D primitives (unit-free)
# ---------------------------------------------------------------------------


def _arc_primitive(t: float, rho: float) -> float:
    """Antiderivative of sqrt(rho^2 - t^2) on [-rho, rho]."""
    t = min(max(t, -rho), rho)
    return 0.5 * (t * math.sqrt(max(rho * rho - t * t, 0.0))
                  + rho * rho * math.asin(t / rho))


def disk_rect_area(rho: float, y0: float, y1: float, z0: float, z1: float) -> float:
    """Area of {(y,z) in [y0,y1]x[z0,z1] : y^2 + z^2 < rho^2}.

    Written as the integral over y of the chord length
    |[z0,z1] intersect (-s(y), s(y))|, s(y) = sqrt(rho^2 - y^2).  Between
    the breakpoints (y = +-rho and the y where s(y) = |z0| or |z1|) each end
    of the chord is either a rectangle side or the circle, so each piece is
    integrated exactly.
    """
    if rho <= 0.0:
        return 0.0
    lo, hi = max(y0, -rho), min(y1, rho)
    if hi <= lo:
        return 0.0
    cuts = {lo, hi}
    for z in (z0, z1):
        if abs(z) < rho:
            w = math.sqrt(rho * rho - z * z)
            for c in (-w, w):
                if lo < c < hi:
                    cuts.add(c)
    pts = sorted(cuts)
    total = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        m = 0.5 * (a + b)
        s = math.sqrt(max(rho * rho - m * m, 0.0))
        top_arc = s < z1
        bot_arc = -s > z0
        top = s if top_arc else z1
        bot = -s if bot_arc else z0
        if top <= bot:
            continue
        arc = _arc_primitive(b, rho) - _arc_primitive(a, rho)
        upper = arc if top_arc else z1 * (b - a)
        lower = -arc if bot_arc else z0 * (b - a)
        total += upper - lower
    return total


def interval_overlap(a0: float, a1: float, b0: float, b1: float) -> float:
    """Length of [a0,a1] intersect (b0,b1)."""
    return max(0.0, min(a1, b1) - max(a0, b0))


# ---------------------------------------------------------------------------
# Geometries.  Each offers, in physical units:
#   edge_len(axis, lo, hi, p)       length of {p + t e_axis, t in [lo,hi]} in Omega
#   face_area(axis, c, lo2, hi2)    area of the axis-normal face at coordinate c
#                                   over the rectangle lo2..hi2 (other two axes
#                                   in increasing order)
#   cell_vol(lo3, hi3)              volume of the box in Omega
#   classify(lo3, hi3)              1 box inside Omega, 0 disjoint, -1 cut
# ---------------------------------------------------------------------------

_OTHER = {0: (1, 2), 1: (0, 2), 2: (0, 1)}

ZERO_FRACTION = 1e-12


def quad_pieces(f, lo: float, hi: float, pts) -> float:
    """Integral of f over [lo, hi], piecewise between the sorted breakpoints
    pts; each piece [a, b] is split at its midpoint m and integrated as
    int_0^sqrt(m-a) f(a + s^2) 2s ds + int_0^sqrt(b-m) f(b - s^2) 2s ds, which
    is smooth in s where f has a square-root endpoint behaviour."""
    cuts = [lo] + sorted(p for p in pts if lo < p < hi) + [hi]
    total = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        if not b > a:
            continue
        m = 0.5 * (a + b)
        left, _ = integrate.quad(lambda s: f(a + s * s) * 2.0 * s, 0.0, math.sqrt(m - a),
                                 epsabs=1e-18, epsrel=1e-13, limit=200)
        right, _ = integrate.quad(lambda s: f(b - s * s) * 2.0 * s, 0.0, math.sqrt(b - m),
                                  epsabs=1e-18, epsrel=1e-13, limit=200)
        total += left + right
    return total


def _clean(x: float) -> float:
    return x if x >= ZERO_FRACTION else 0.0


@dataclass
class Box:
    """The whole domain box is the cavity (only the walls conduct)."""

    def classify(self, lo, hi):
        return 1

    def edge_len(self, axis, lo, hi, p):
        return hi - lo

    def face_area(self, axis, c, lo2, hi2):
        return (hi2[0] - lo2[0]) * (hi2[1] - lo2[1])

    def cell_vol(self, lo3, hi3):
        return float(np.prod(np.subtract(hi3, lo3)))


@dataclass
class Ellipsoid:
    """Open axis-aligned ellipsoid sum(((x_a - c_a)/s_a)^2) < 1.

    A sphere is the case s_x = s_y = s_z = R.  Each quantity is computed in
    the scaled coordinates u_a = (x_a - c_a)/s_a, where Omega is the unit
    ball, and mapped back with the Jacobian of the scaling.
    """

    center: tuple
    semi: tuple

    def _u(self, a, x):
        return (x - self.center[a]) / self.semi[a]

    def classify(self, lo, hi):
        ulo = [self._u(a, lo[a]) for a in range(3)]
        uhi = [self._u(a, hi[a]) for a in range(3)]
        far = sum(max(abs(ulo[a]), abs(uhi[a])) ** 2 for a in range(3))
        if far < 1.0:
            return 1
        near = 0.0
        for a in range(3):
            if ulo[a] > 0.0:
                near += ulo[a] ** 2
            elif uhi[a] < 0.0:
                near += uhi[a] ** 2
        if near >= 1.0:
            return 0
        return -1

    def edge_len(self, axis, lo, hi, p):
        d2 = sum(self._u(a, p[a]) ** 2 for a in range(3) if a != axis)
        if d2 >= 1.0:
            return 0.0
        s = math.sqrt(1.0 - d2) * self.semi[axis]
        c = self.center[axis]
        return interval_overlap(lo, hi, c - s, c + s)

    def _section_area_u(self, axis, uc, ulo2, uhi2):
        rho2 = 1.0 - uc * uc
        if rho2 <= 0.0:
            return 0.0
        return disk_rect_area(math.sqrt(rho2), ulo2[0], uhi2[0], ulo2[1], uhi2[1])

    def face_area(self, axis, c, lo2, hi2):
        b, d = _OTHER[axis]
        ulo2 = (self._u(b, lo2[0]), self._u(d, lo2[1]))
        uhi2 = (self._u(b, hi2[0]), self._u(d, hi2[1]))
        return (self._section_area_u(axis, self._u(axis, c), ulo2, uhi2)
                * self.semi[b] * self.semi[d])

    def cell_vol(self, lo3, hi3):
        ulo = [self._u(a, lo3[a]) for a in range(3)]
        uhi = [self._u(a, hi3[a]) for a in range(3)]
        # kinks of the x-section area: where the section radius
        # rho(ux) = sqrt(1-ux^2) equals a distance to a side line or corner
        dists = [abs(ulo[1]), abs(uhi[1]), abs(ulo[2]), abs(uhi[2])]
        dists += [math.hypot(y, z) for y in (ulo[1], uhi[1]) for z in (ulo[2], uhi[2])]
        dists.append(0.0)
        pts = set()
        for d in dists:
            if d < 1.0:
                r = math.sqrt(1.0 - d * d)
                for q in (-r, r):
                    if ulo[0] < q < uhi[0]:
                        pts.add(q)

        def area(ux):
            return self._section_area_u(0, ux, (ulo[1], ulo[2]), (uhi[1], uhi[2]))

        # the section radius has a square-root end behaviour at the poles
        # (ux -> +-1) and where it meets a distance: integrated piecewise with
        # the end substitution of quad_pieces
        val = quad_pieces(area, ulo[0], uhi[0], pts)
        return val * self.semi[0] * self.semi[1] * self.semi[2]


def sphere(center=(0.5, 0.5, 0.5), radius=0.45) -> Ellipsoid:
    return Ellipsoid(tuple(center), (radius, radius, radius))


@dataclass
class EllipticCells:
    """Open body of revolution about the z-line through (ax, ay): a tube of
    radius r_iris and length `tube`, `ncell` cells whose radius rises along
    an elliptic arc from r_iris at both cell ends to r_eq at the cell middle,
    and a second tube; conducting end plates at z0 and z0 + 2 tube + ncell L.
    (A synthetic stand-in for the multi-cell accelerator cavity of Sec. 6.3,
    whose real profile the paper does not give.)"""

    axis: tuple
    z0: float
    ncell: int
    r_eq: float
    r_iris: float
    L: float
    tube: float

    @property
    def z_end(self):
        return self.z0 + 2 * self.tube + self.ncell * self.L

    def centres(self):
        c0 = self.z0 + self.tube
        return [c0 + (m + 0.5) * self.L for m in range(self.ncell)]

    def junctions(self):
        c0 = self.z0 + self.tube
        return [self.z0, self.z_end] + [c0 + m * self.L for m in range(self.ncell + 1)]

    def radius(self, z):
        if not (self.z0 < z < self.z_end):
            return 0.0
        for zc in self.centres():
            t = (z - zc) / (0.5 * self.L)
            if abs(t) < 1.0:
                return self.r_iris + (self.r_eq - self.r_iris) * math.sqrt(1.0 - t * t)
        return self.r_iris

    def above(self, R):
        """Intervals of z where radius(z) > R (R >= 0)."""
        out = []
        c0 = self.z0 + self.tube
        if R < self.r_iris:
            return [(self.z0, self.z_end)]
        if R >= self.r_eq:
            return out
        t = (R - self.r_iris) / (self.r_eq - self.r_iris)
        half = 0.5 * self.L * math.sqrt(1.0 - t * t)
        for zc in self.centres():
            out.append((zc - half, zc + half))
        return out

    def crossings(self, R):
        """z where radius(z) passes through R."""
        pts = []
        for a, b in self.above(R):
            pts += [a, b]
        return pts

    def _rlim(self, z):
        """radius(z), with the tube radius as the limit at the end plates"""
        if z <= self.z0 or z >= self.z_end:
            return self.r_iris
        return self.radius(z)

    def _rmin_rmax(self, zlo, zhi):
        """Bounds of radius(z) over [zlo, zhi] intersect (z0, z_end): the
        profile is monotone between a junction and the next cell middle."""
        a, b = max(zlo, self.z0), min(zhi, self.z_end)
        zs = [a, b] + [z for z in self.junctions() if a < z < b]
        rs = [self._rlim(z) for z in zs]
        rmax = max(rs + [self.r_eq for zc in self.centres() if a < zc < b])
        return min(rs), rmax

    def classify(self, lo, hi):
        ax, ay = self.axis
        dx = [lo[0] - ax, hi[0] - ax]
        dy = [lo[1] - ay, hi[1] - ay]
        far = math.sqrt(max(d * d for d in dx) + max(d * d for d in dy))
        nx = 0.0 if dx[0] <= 0.0 <= dx[1] else min(abs(dx[0]), abs(dx[1]))
        ny = 0.0 if dy[0] <= 0.0 <= dy[1] else min(abs(dy[0]), abs(dy[1]))
        near = math.hypot(nx, ny)
        if hi[2] <= self.z0 or lo[2] >= self.z_end:
            return 0
        rmin, rmax = self._rmin_rmax(lo[2], hi[2])
        if near >= rmax:
            return 0
        if far < rmin and lo[2] > self.z0 and hi[2] < self.z_end:
            return 1
        return -1

    def edge_len(self, axis, lo, hi, p):
        ax, ay = self.axis
        if axis == 2:
            rho = math.hypot(p[0] - ax, p[1] - ay)
            return sum(interval_overlap(lo, hi, a, b) for a, b in self.above(rho))
        r = self.radius(p[2])
        other = p[1] - ay if axis == 0 else p[0] - ax
        if r <= abs(other):
            return 0.0
        s = math.sqrt(r * r - other * other)
        c = ax if axis == 0 else ay
        return interval_overlap(lo, hi, c - s, c + s)

    def face_area(self, axis, c, lo2, hi2):
        ax, ay = self.axis
        if axis == 2:
            return disk_rect_area(self.radius(c), lo2[0] - ax, hi2[0] - ax, lo2[1] - ay, hi2[1] - ay)
        # x-face (axis 0): coordinates (y, z); y-face (axis 1): (x, z)
        d = c - (ax if axis == 0 else ay)
        cen = ay if axis == 0 else ax
        t0, t1 = lo2[0] - cen, hi2[0] - cen
        zlo, zhi = lo2[1], hi2[1]

        def chord(z):
            r = self.radius(z)
            if r <= abs(d):
                return 0.0
            s = math.sqrt(r * r - d * d)
            return interval_overlap(t0, t1, -s, s)

        pts = set(z for z in self.junctions() if zlo < z < zhi)
        for R in (abs(d), math.hypot(d, t0), math.hypot(d, t1)):
            pts.update(z for z in self.crossings(R) if zlo < z < zhi)
        return quad_pieces(chord, zlo, zhi, pts)

    def cell_vol(self, lo3, hi3):
        ax, ay = self.axis
        x0, x1, y0, y1 = lo3[0] - ax, hi3[0] - ax, lo3[1] - ay, hi3[1] - ay
        zlo, zhi = lo3[2], hi3[2]

        def area(z):
            return disk_rect_area(self.radius(z), x0, x1, y0, y1)

        dists = {abs(x0), abs(x1), abs(y0), abs(y1)}
        dists.update(math.hypot(x, y) for x in (x0, x1) for y in (y0, y1))
        pts = set(z for z in self.junctions() if zlo < z < zhi)
        for R in dists:
            pts.update(z for z in self.crossings(R) if zlo < z < zhi)
        return quad_pieces(area, zlo, zhi, pts)


def nine_cell(axis=(0.0, 0.0), z0=0.0, ncell=9, r_eq=0.103, r_iris=0.035, L=0.115, tube=0.1):
    """The synthetic 9-cell elliptic cavity (equator 0.103, iris 0.035, cells
    0.115 long, 0.1 end tubes)."""
    return EllipticCells(tuple(axis), z0, ncell, r_eq, r_iris, L, tube)


def bor_volume(g: EllipticCells):
    """Exact volume of the body: pi * integral of r(z)^2."""
    v = 2 * g.tube * math.pi * g.r_iris ** 2
    a, b = g.r_iris, g.r_eq - g.r_iris
    # one cell: integral over the length L of (a + b sqrt(1-t^2))^2 with z = t L/2
    cell = 0.5 * g.L * (2 * a * a + math.pi * a * b + (4.0 / 3.0) * b * b)
    return v + g.ncell * math.pi * cell


# ---------------------------------------------------------------------------
# Fraction arrays on the Yee grid
# ---------------------------------------------------------------------------

FACE_SHAPES = {
    "ax": lambda n: (n[2], n[1], n[0] + 1),
    "ay": lambda n: (n[2], n[1] + 1, n[0]),
    "az": lambda n: (n[2] + 1, n[1], n[0]),
}
EDGE_SHAPES = {
    "lx": lambda n: (n[2] + 1, n[1] + 1, n[0]),
    "ly": lambda n: (n[2] + 1, n[1], n[0] + 1),
    "lz": lambda n: (n[2], n[1] + 1, n[0] + 1),
}


def face_fraction(geom, n, h, axis, i, j, k, origin=(0, 0, 0)) -> float:
    """Area fraction of the axis-normal face with low corner node (i,j,k);
    the node's coordinates are (index + origin) h (walls: indices 0, n)."""
    idx = (i, j, k)
    if idx[axis] == 0 or idx[axis] == n[axis]:
        return 0.0  # face lies in a conducting wall of the domain
    idx = tuple(x + o for x, o in zip(idx, origin))
    b, d = _OTHER[axis]
    c = idx[axis] * h
    lo2 = (idx[b] * h, idx[d] * h)
    hi2 = ((idx[b] + 1) * h, (idx[d] + 1) * h)
    lo3 = [x * h for x in idx]
    hi3 = list(lo3)
    hi3[b] += h
    hi3[d] += h
    cls = geom.classify(lo3, hi3)
    if cls == 1:
        return 1.0
    if cls == 0:
        return 0.0
    return _clean(geom.face_area(axis, c, lo2, hi2) / (h * h))


def edge_fraction(geom, n, h, axis, i, j, k, origin=(0, 0, 0)) -> float:
    """Length fraction of the axis-directed edge starting at node (i,j,k)."""
    idx = (i, j, k)
    for a in _OTHER[axis]:
        if idx[a] == 0 or idx[a] == n[a]:
            return 0.0  # edge lies in a conducting wall of the domain
    idx = tuple(x + o for x, o in zip(idx, origin))
    p = [x * h for x in idx]
    lo = idx[axis] * h
    return _clean(geom.edge_len(axis, lo, lo + h, p) / h)


def cell_fraction(geom, n, h, i, j, k, origin=(0, 0, 0)) -> float:
    i, j, k = i + origin[0], j + origin[1], k + origin[2]
    lo3 = [i * h, j * h, k * h]
    hi3 = [(i + 1) * h, (j + 1) * h, (k + 1) * h]
    cls = geom.classify(lo3, hi3)
    if cls == 1:
        return 1.0
    if cls == 0:
        return 0.0
    return _clean(geom.cell_vol(lo3, hi3) / h ** 3)


def _classify_all(geom, lo, hi):
    """Vectorised ``classify`` over arrays of boxes (lo, hi: (m, 3))."""
    if isinstance(geom, Box):
        return np.ones(lo.shape[0], dtype=int)
    if isinstance(geom, Ellipsoid):
        c = np.asarray(geom.center)
        s = np.asarray(geom.semi)
        ulo = (lo - c) / s
        uhi = (hi - c) / s
        far = np.sum(np.maximum(abs(ulo), abs(uhi)) ** 2, axis=1)
        near = np.sum(np.where(ulo > 0, ulo, np.where(uhi < 0, uhi, 0.0)) ** 2, axis=1)
        return np.where(far < 1.0, 1, np.where(near >= 1.0, 0, -1))
    return np.array([geom.classify(a, b) for a, b in zip(lo, hi)])


def _family(shape):
    k, j, i = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]),
                          np.arange(shape[2]), indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def face_fractions(geom, n, h, axis, origin=(0, 0, 0)) -> np.ndarray:
    """Area fractions of all axis-normal faces (array [k, j, i])."""
    n = tuple(int(x) for x in n)
    shape = FACE_SHAPES[("ax", "ay", "az")[axis]](n)
    idx = _family(shape)
    b, d = _OTHER[axis]
    lo = (idx + np.asarray(origin)) * h
    hi = lo.copy()
    hi[:, b] += h
    hi[:, d] += h
    cls = _classify_all(geom, lo.astype(float), hi.astype(float)).astype(float)
    wall = (idx[:, axis] == 0) | (idx[:, axis] == n[axis])
    cls[wall] = 0.0
    out = cls.copy()
    for m in np.flatnonzero(cls < 0):
        i, j, k = (int(x) for x in idx[m])
        out[m] = face_fraction(geom, n, h, axis, i, j, k, origin)
    return out.reshape(shape)


def edge_fractions(geom, n, h, axis, origin=(0, 0, 0)) -> np.ndarray:
    n = tuple(int(x) for x in n)
    shape = EDGE_SHAPES[("lx", "ly", "lz")[axis]](n)
    out = np.zeros(shape)
    for (k, j, i), _ in np.ndenumerate(out):
        out[k, j, i] = edge_fraction(geom, n, h, axis, i, j, k, origin)
    return out


def cell_fractions(geom, n, h, origin=(0, 0, 0)) -> np.ndarray:
    n = tuple(int(x) for x in n)
    shape = (n[2], n[1], n[0])
    idx = _family(shape)
    lo = ((idx + np.asarray(origin)) * h).astype(float)
    cls = _classify_all(geom, lo, lo + h).astype(float)
    out = cls.copy()
    for m in np.flatnonzero(cls < 0):
        i, j, k = (int(x) for x in idx[m])
        out[m] = cell_fraction(geom, n, h, i, j, k, origin)
    return out.reshape(shape)


def _either_side(mask, np_axis, pad_value):
    """For an array of items along np_axis (length N), the items' boundary
    positions 0..N: True where the item on either side is True."""
    pad = [(0, 0)] * 3
    pad[np_axis] = (1, 1)
    e = np.pad(mask, pad, constant_values=pad_value)
    lo = np.take(e, np.arange(0, e.shape[np_axis] - 1), axis=np_axis)
    hi = np.take(e, np.arange(1, e.shape[np_axis]), axis=np_axis)
    return lo | hi


def drop_faces_of_empty_cells(fr: dict) -> dict:
    """Set a = 0 on every face that has a cell with v = 0 on either side."""
    out = dict(fr)
    empty = fr["v"] == 0.0                                  # (Nz, Ny, Nx)
    for axis, name in enumerate(("ax", "ay", "az")):
        out[name] = np.where(_either_side(empty, 2 - axis, False), 0.0, fr[name])
    return out


def drop_edges_of_zero_faces(fr: dict) -> dict:
    """Set l = 0 on every edge with a face of a = 0 around it.  An edge along
    axis e is bounded by the two faces normal to each other axis b, which lie
    on either side of it along the third axis d."""
    out = dict(fr)
    faces = ("ax", "ay", "az")
    for e, name in enumerate(("lx", "ly", "lz")):
        drop = np.zeros(fr[name].shape, bool)
        for b in range(3):
            if b == e:
                continue
            d = 3 - e - b
            drop |= _either_side(fr[faces[b]] == 0.0, 2 - d, False)
        out[name] = np.where(drop, 0.0, fr[name])
    return out


def fractions(geom, n, h, drop_empty=True, origin=(0, 0, 0)) -> dict:
    """All seven fraction arrays of the grid n = (Nx, Ny, Nz), cell size h;
    with drop_empty, the two consistency rules above are applied.  origin
    (integers): the grid's cell (i,j,k) is [(i+o_x)h, (i+o_x+1)h] x ... --
    a window of a larger grid, with the window's own boundary as its walls;
    its interior entities then have the larger grid's coordinates exactly."""
    out = {}
    for axis, name in enumerate(("ax", "ay", "az")):
        out[name] = face_fractions(geom, n, h, axis, origin)
    for axis, name in enumerate(("lx", "ly", "lz")):
        out[name] = edge_fractions(geom, n, h, axis, origin)
    out["v"] = cell_fractions(geom, n, h, origin)
    return drop_edges_of_zero_faces(drop_faces_of_empty_cells(out)) if drop_empty else out


def count_active_faces(geom, n, h) -> int:
    """Number of faces with a > 0, decided by classification alone (a face
    whose closed rectangle meets the open cavity has positive area)."""
    n = tuple(int(x) for x in n)
    total = 0
    for axis in range(3):
        shape = FACE_SHAPES[("ax", "ay", "az")[axis]](n)
        idx = _family(shape)
        b, d = _OTHER[axis]
        lo = (idx * h).astype(float)
        hi = lo.copy()
        hi[:, b] += h
        hi[:, d] += h
        cls = _classify_all(geom, lo, hi)
        wall = (idx[:, axis] == 0) | (idx[:, axis] == n[axis])
        total += int(np.sum((cls != 0) & ~wall))
    return total


# ---------------------------------------------------------------------------
# General cavities from a sampled level set: tetrahedral cut-cell volumes
# (Sec. 6.1: volumes from tetrahedral subvolumes conforming to the surface)
# ---------------------------------------------------------------------------

def _negative_hull_measure(points, values, dim):
    """Measure (length, area or volume) of the part of a simplex where the
    linear interpolant of `values` at its vertices `points` is negative: the
    convex hull of its negative vertices and of the zero crossings on its
    edges (the negative part of a simplex under a linear function is convex,
    with exactly those vertices).  Computed by Qhull; a flat hull has
    measure 0."""
    from scipy.spatial import ConvexHull, QhullError
    pts = [p for p, v in zip(points, values) if v < 0.0]
    k = len(points)
    for a in range(k):
        for b in range(a + 1, k):
            va, vb = values[a], values[b]
            if (va < 0.0) != (vb < 0.0):
                t = va / (va - vb)
                pts.append(points[a] + t * (points[b] - points[a]))
    if len(pts) < dim + 1:
        return 0.0
    pts = np.array(pts)
    if dim == 1:
        return float(pts[:, 0].max() - pts[:, 0].min())
    try:
        return float(ConvexHull(pts).volume)
    except QhullError:
        return 0.0


def levelset_fractions(phi, s, n, drop_empty=True) -> dict:
    """Cut fractions of {phi_lin < 0} for phi sampled on the nodes of the grid
    n = (Nx, Ny, Nz) refined s times per cell (array [K, J, I] of shape
    (s Nz + 1, s Ny + 1, s Nx + 1)), phi_lin the linear interpolant on the
    Kuhn tetrahedra of the refined lattice (6 per refined cube along its
    main diagonal; each refined square split along the diagonal through its
    lowest and highest corner).  Units are cells; all walls conduct.  Every
    cut simplex is measured as a convex hull (``_negative_hull_measure``)."""
    nx, ny, nz = n
    out = {name: np.zeros(shape(n)) for name, shape in FACE_SHAPES.items()}
    out.update({name: np.zeros(shape(n)) for name, shape in EDGE_SHAPES.items()})
    out["v"] = np.zeros((nz, ny, nx))

    def val(I, J, K):
        return phi[K, J, I]

    unit = np.eye(3)
    # cells: 6 tetrahedra per refined cube
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                block = phi[k * s:(k + 1) * s + 1, j * s:(j + 1) * s + 1, i * s:(i + 1) * s + 1]
                if block.max() < 0.0:
                    out["v"][k, j, i] = 1.0
                    continue
                if block.min() >= 0.0:
                    continue
                vol = 0.0
                for cz in range(s):
                    for cy in range(s):
                        for cx in range(s):
                            corner = np.array([cx, cy, cz], float)
                            for pm in perms:
                                verts = [corner, corner + unit[pm[0]], corner + unit[pm[0]] + unit[pm[1]],
                                         corner + 1.0]
                                vals = [block[int(v[2]), int(v[1]), int(v[0])] for v in verts]
                                vol += _negative_hull_measure(verts, vals, 3)
                out["v"][k, j, i] = vol / s ** 3
    # faces normal to axis a, over the other two axes b < d
    for a, name in enumerate(("ax", "ay", "az")):
        b, d = [x for x in range(3) if x != a]
        arr = out[name]
        for idx in np.ndindex(arr.shape):
            kk, jj, ii = idx
            cell = (ii, jj, kk)
            if cell[a] == 0 or cell[a] == n[a]:
                continue
            area = 0.0
            for u in range(s):
                for w in range(s):
                    corners = []
                    for q in range(4):
                        node = [cell[0] * s, cell[1] * s, cell[2] * s]
                        node[b] += u + (q & 1)
                        node[d] += w + (q >> 1)
                        corners.append((np.array([u + (q & 1), w + (q >> 1)], float), val(*node)))
                    for tri in ((0, 1, 3), (0, 2, 3)):
                        area += _negative_hull_measure([corners[t][0] for t in tri], [corners[t][1] for t in tri], 2)
            arr[idx] = area / s ** 2
    # edges along axis a
    for a, name in enumerate(("lx", "ly", "lz")):
        b, d = [x for x in range(3) if x != a]
        arr = out[name]
        for idx in np.ndindex(arr.shape):
            kk, jj, ii = idx
            node0 = (ii, jj, kk)
            if node0[b] in (0, n[b]) or node0[d] in (0, n[d]):
                continue
            length = 0.0
            for u in range(s):
                p0 = [node0[0] * s, node0[1] * s, node0[2] * s]
                p1 = list(p0)
                p0[a] += u
                p1[a] += u + 1
                length += _negative_hull_measure([np.array([0.0]), np.array([1.0])], [val(*p0), val(*p1)], 1)
            arr[idx] = length / s
    for name in out:
        out[name] = np.where(out[name] >= 1e-12, out[name], 0.0)
    return drop_edges_of_zero_faces(drop_faces_of_empty_cells(out)) if drop_empty else out


def sample_levelset(fun, n, h, s):
    """phi on the nodes of the grid refined s times: fun(x, y, z) at
    (I, J, K) h / s, array [K, J, I]."""
    nx, ny, nz = n
    K, J, I = np.meshgrid(np.arange(s * nz + 1), np.arange(s * ny + 1), np.arange(s * nx + 1), indexing="ij")
    return fun(I * h / s, J * h / s, K * h / s)
