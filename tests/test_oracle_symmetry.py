"""Pins of the 9-cell geometry and of the PMC symmetry-plane oracle.

* elliptic-cell body of revolution: the volume sum equals pi * integral of
  r(z)^2 in closed form, also layer by layer with the junctions (irises,
  where r(z) has a vertical tangent) inside cells; every z-plane sum of face
  areas is the disk area;
  every z-line sum of edge lengths is the measure of {r(z) > rho};
* the library's quarter-cavity fractions (axis on the corner, PMC planes)
  equal the oracle's full-cavity fractions on that quarter, and its ghost
  layer is their mirror image;
* PMC restriction (Sec. 6.3 quarter runs): Q^T M Q = diag(mult) R M Q, and
  the symmetric pencil's eigenvalues are eigenvalues of the full cavity.
"""
import math

import numpy as np
import pytest

from oracle import eigs, geometry as geo, symmetry as sym
import layout as lay

# a small two-cell cavity that a 16 x 16 x 24 full grid (h = 1/16) holds
SMALL = dict(ncell=2, r_eq=0.4, r_iris=0.18, L=0.5, tube=0.25)
H = 1.0 / 16


def small_bor(axis):
    return geo.EllipticCells(tuple(axis), 0.0, SMALL["ncell"], SMALL["r_eq"], SMALL["r_iris"],
                             SMALL["L"], SMALL["tube"])


@pytest.fixture(scope="module")
def full_small():
    n = (16, 16, 24)
    g = small_bor((8 * H, 8 * H))
    return g, n, geo.fractions(g, n, H)


def test_bor_volume_closed_form():
    g = geo.nine_cell()
    assert geo.bor_volume(g) == pytest.approx(0.0269322, abs=5e-8)


def test_bor_measure_sums(full_small):
    g, n, _ = full_small
    fr = geo.fractions(g, n, H, drop_empty=False)
    assert fr["v"].sum() * H ** 3 == pytest.approx(geo.bor_volume(g), rel=1e-12)
    for k in range(1, n[2]):
        r = g.radius(k * H)
        assert fr["az"][k].sum() * H * H == pytest.approx(math.pi * r * r, abs=1e-13)
    for j in range(0, n[1] + 1, 3):
        for i in range(0, n[0] + 1, 3):
            rho = math.hypot(i * H - 8 * H, j * H - 8 * H)
            want = sum(b - a for a, b in g.above(rho)) if (0 < i < n[0] and 0 < j < n[1]) else 0.0
            assert fr["lz"][:, j, i].sum() * H == pytest.approx(want, abs=1e-13)


def layer_volume(g, z_lo, z_hi):
    """pi * integral of r(z)^2 over [z_lo, z_hi], in closed form and in
    40-digit arithmetic (the difference of two primitives near t = 1 cancels
    most digits in double): tubes give r_iris^2; on a cell, with
    z = zc + t L/2 and r = a + b sqrt(1 - t^2), the primitive of r^2 in t is
    a^2 t + a b (t sqrt(1-t^2) + asin t) + b^2 (t - t^3/3)."""
    mpmath = pytest.importorskip("mpmath")
    mp = mpmath.mp
    mp.dps = 40
    F = mpmath.mpf
    a, b = F(g.r_iris), F(g.r_eq) - F(g.r_iris)

    def prim(t):
        t = min(F(1), max(F(-1), t))
        return a * a * t + a * b * (t * mpmath.sqrt(1 - t * t) + mpmath.asin(t)) + b * b * (t - t ** 3 / 3)

    lo, hi = max(F(z_lo), F(g.z0)), min(F(z_hi), F(g.z_end))
    if hi <= lo:
        return F(0)
    c0 = F(g.z0) + F(g.tube)
    c1 = c0 + g.ncell * F(g.L)
    tube = max(F(0), min(hi, c0) - lo) + max(F(0), hi - max(lo, c1))
    total = tube * a * a
    for m in range(g.ncell):
        zc = c0 + (m + F(0.5)) * F(g.L)
        t0, t1 = (lo - zc) / (F(g.L) / 2), (hi - zc) / (F(g.L) / 2)
        if t1 > -1 and t0 < 1:
            total += F(g.L) / 2 * (prim(t1) - prim(t0))
    return mpmath.pi * total


def test_bor_layer_volumes_with_junctions_inside_cells():
    """Small two-cell body shifted so that its junctions fall inside cells."""
    n = (16, 16, 25)
    g = geo.EllipticCells((8 * H, 8 * H), 0.37 * H, SMALL["ncell"], SMALL["r_eq"], SMALL["r_iris"],
                          SMALL["L"], SMALL["tube"])
    fr = geo.fractions(g, n, H, drop_empty=False)
    assert all(abs(z / H - round(z / H)) > 0.1 for z in g.junctions())
    for k in range(n[2]):
        want = float(layer_volume(g, k * H, (k + 1) * H) / H ** 3)
        assert math.fsum(fr["v"][k].ravel()) == pytest.approx(want, abs=2e-13), k


def test_nine_cell_iris_layer_volume():
    """The 9-cell iris at the 1024-cell resolution: the radius rises by ~11
    cells within one cell of the iris (vertical tangent), the case where an
    adaptive rule in z stalls.  A quarter of the cross-section (axis on the
    grid corner), the one layer that holds the iris; ~700 cut cells, so the
    bar 1e-11 (cell units) leaves room for their rounding."""
    h = 1.235 / 1024
    z_iris = 0.1 + 3 * 0.115
    g = geo.nine_cell(axis=(0.0, 0.0), z0=0.43 * h - z_iris)   # this iris at z = 0.43 h
    n = (56, 56, 1)
    assert [round(z / h, 6) for z in g.junctions() if 0 < z < h] == [0.43]
    fr = geo.fractions(g, n, h, drop_empty=False)
    assert g.radius(0.0) < n[0] * h and g.radius(h) < n[0] * h
    want = float(layer_volume(g, 0.0, h) / 4 / h ** 3)
    assert math.fsum(fr["v"][0].ravel()) == pytest.approx(want, abs=1e-11)


def test_library_quarter_fractions_match_oracle(full_small):
    from paper_1301_3794_amd import dm
    g, n, fr = full_small
    ext = sym.MirrorExtension((8, 8, 24), H, (0, 1))
    ref = lay.fractions_to_padded(ext.half_fractions(fr), (8, 8, 24))
    pg = dm.elliptic_bor((0.0, 0.0), 0.0, SMALL["ncell"], SMALL["r_eq"], SMALL["r_iris"],
                         SMALL["L"], SMALL["tube"], bc_lo=(dm.BC_PMC, dm.BC_PMC, dm.BC_PEC))
    got = dm.compute_fractions(pg, (8, 8, 24), H)
    inner = lay.fractions_to_padded({s: np.ones_like(v) for s, v in ext.half_fractions(fr).items()},
                                    (8, 8, 24)) > 0
    assert np.max(abs(got[inner] - ref[inner])) <= 1e-13
    # ghost layer at i = -1: the mirror image across x = 0
    a = got.reshape(7, 26, 10, 10)
    assert np.max(abs(a[0][1:25, 1:9, 0] - a[0][1:25, 1:9, 2])) == 0.0   # ax: node-centred
    assert np.max(abs(a[1][1:25, 1:9, 0] - a[1][1:25, 1:9, 1])) == 0.0   # ay: cell-centred
    assert np.max(abs(a[6][1:25, 1:9, 0] - a[6][1:25, 1:9, 1])) == 0.0   # v


def test_pmc_restriction_algebra_and_spectrum(full_small):
    g, n, fr = full_small
    ext = sym.MirrorExtension((8, 8, 24), H, (0, 1))
    hop = sym.HalfOperators(ext, fr, 2.0)
    lhs = (ext.Q.T @ hop.full.M @ ext.Q)
    rhs = sym.sp.diags(ext.mult) @ hop.M_rows
    assert abs(lhs - rhs).max() <= 1e-12 * abs(lhs).max()
    assert set(np.unique(ext.mult)) == {2.0, 4.0}
    w_sym, _ = sym.sym_dense_eigs(hop, 8)
    w_full, _ = eigs.lanczos_eigs(hop.full, 24, sigma_o=2.0, block=4, tol=1e-11)[:2]
    inside = w_sym[w_sym < w_full.max()]
    assert inside.size >= 5
    for w in inside:
        assert np.min(abs(w_full - w) / w) <= 1e-10
