"""Pins of the 9-cell geometry and of the PMC symmetry-plane oracle.

* elliptic-cell body of revolution: the volume sum equals pi * integral of
  r(z)^2 in closed form; every z-plane sum of face areas is the disk area;
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
