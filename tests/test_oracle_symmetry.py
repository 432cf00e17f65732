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


def profile_radius_crossings(g, R):
    """z where the profile's radius equals R, from the profile's definition
    (cells: R = r_iris + (r_eq - r_iris) sqrt(1 - t^2), z = zc + t L/2),
    written out here independently of the oracle's helpers."""
    if not (g.r_iris < R < g.r_eq):
        return []
    t = math.sqrt(1.0 - ((R - g.r_iris) / (g.r_eq - g.r_iris)) ** 2)
    c0 = g.z0 + g.tube
    out = []
    for m in range(g.ncell):
        zc = c0 + (m + 0.5) * g.L
        out += [zc - t * g.L / 2, zc + t * g.L / 2]
    return out


def plane_section_area(g, d):
    """Area of the body's section by a plane at distance d from the axis,
    parallel to it: the integral over z of the full chord 2 sqrt(r(z)^2 - d^2)
    (40-digit quadrature, split at the profile's junctions and at the z
    where r(z) = d)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    c0 = g.z0 + g.tube
    cuts = sorted(set([g.z0, c0 + g.ncell * g.L, g.z_end] + [c0 + m * g.L for m in range(g.ncell + 1)]
                      + profile_radius_crossings(g, d)))

    def f(z):
        r = mpmath.mpf(g.r_iris)
        for m in range(g.ncell):
            zc = c0 + (m + 0.5) * g.L
            t = (z - zc) / (mpmath.mpf(g.L) / 2)
            if abs(t) < 1:
                r = g.r_iris + (g.r_eq - g.r_iris) * mpmath.sqrt(1 - t * t)
        q = r * r - mpmath.mpf(d) ** 2
        return 2 * mpmath.sqrt(q) if q > 0 else mpmath.mpf(0)
    return float(sum(mpmath.quad(f, [a, b]) for a, b in zip(cuts[:-1], cuts[1:])))


def test_bor_xy_face_plane_sums_and_edge_line_sums(full_small):
    """x- and y-faces: every interior node plane's area sum is the plane
    section of the body; x- and y-edges: every interior line's length sum is
    the chord of the disk r(z) at that line's offset from the axis."""
    g, n, _ = full_small
    fr = geo.fractions(g, n, H, drop_empty=False)
    for i in range(1, n[0]):
        d = abs(i * H - 8 * H)
        assert math.fsum(fr["ax"][:, :, i].ravel()) * H * H == pytest.approx(plane_section_area(g, d), abs=1e-12)
    for j in range(1, n[1], 2):
        d = abs(j * H - 8 * H)
        assert math.fsum(fr["ay"][:, j, :].ravel()) * H * H == pytest.approx(plane_section_area(g, d), abs=1e-12)
    for k in range(1, n[2]):
        r = g.radius(k * H)
        for j in range(1, n[1]):
            dy = j * H - 8 * H
            want = 2.0 * math.sqrt(r * r - dy * dy) if r > abs(dy) else 0.0
            assert math.fsum(fr["lx"][k, j, :]) * H == pytest.approx(want, abs=1e-13)
        for i in range(1, n[0], 3):
            dx = i * H - 8 * H
            want = 2.0 * math.sqrt(r * r - dx * dx) if r > abs(dx) else 0.0
            assert math.fsum(fr["ly"][k, :, i]) * H == pytest.approx(want, abs=1e-13)


def test_bor_cut_xy_faces_vs_2d_quadrature():
    """Sampled cut x- and y-faces of the 9-cell body at a coarse grid (iris
    cusps inside faces) against SciPy's adaptive 2-D quadrature of the
    indicator {(t - axis)^2 + d^2 < r(z)^2} over the face (no breakpoints
    given)."""
    from scipy import integrate
    h = 1.235 / 128
    g = geo.nine_cell(axis=(12 * h, 12 * h))
    n = (24, 24, 128)
    rng = np.random.default_rng(3)
    checked = 0
    while checked < 16:
        axis = int(rng.integers(0, 2))
        i = int(rng.integers(1, n[axis]))
        t_idx = int(rng.integers(0, n[1 - axis]))
        k = int(rng.integers(0, n[2]))
        idx = [0, 0, k]
        idx[axis], idx[1 - axis] = i, t_idx
        a = geo.face_fraction(g, n, h, axis, *idx)
        if not 0.0 < a < 1.0:
            continue
        d = i * h - 12 * h
        t0, t1 = t_idx * h - 12 * h, (t_idx + 1) * h - 12 * h

        def lo(z):
            r = g.radius(z)
            s = math.sqrt(max(r * r - d * d, 0.0))
            return min(max(-s, t0), t1)

        def hi(z):
            r = g.radius(z)
            s = math.sqrt(max(r * r - d * d, 0.0))
            return max(min(s, t1), t0)
        ref, _ = integrate.dblquad(lambda t, z: 1.0, k * h, (k + 1) * h, lo, hi, epsabs=1e-13, epsrel=1e-11)
        assert a == pytest.approx(ref / (h * h), abs=1e-9), (axis, idx)
        checked += 1


@pytest.fixture(scope="module")
def half_small(full_small):
    g, n, fr = full_small
    vc = sym.HalfVCycle(fr, (8, 8, 24), H, 2.0, (0, 1), 3)
    return fr, vc


def test_half_vcycle_is_self_adjoint(half_small):
    """B_h diag(1/mult) is symmetric on the active half faces (B_h
    approximates (R M Q)^-1 = (diag(1/mult) Q^T M Q)^-1, so this is the
    V-cycle's symmetry for the symmetric pencil); a transposed transfer or a
    smoothing order that is not reversed on the way up breaks it."""
    fr, vc = half_small
    hop = vc.levels[0].op
    act = hop.act
    mult = hop.ext.mult
    rng = np.random.default_rng(1)
    x, y = np.zeros(hop.grid.n_faces), np.zeros(hop.grid.n_faces)
    x[act], y[act] = rng.standard_normal(act.size), rng.standard_normal(act.size)
    u = x @ vc(y / mult)
    w = y @ vc(x / mult)
    assert abs(u - w) <= 1e-12 * max(abs(u), abs(w))


def test_half_vcycle_contracts(half_small):
    """The error propagator I - B_h (R M Q) on the half cavity has spectral
    radius well below 1 (power iteration)."""
    fr, vc = half_small
    hop = vc.levels[0].op
    act = hop.act
    e = np.zeros(hop.grid.n_faces)
    e[act] = np.random.default_rng(2).standard_normal(act.size)
    rho = 0.0
    for _ in range(30):
        e_new = e - vc(hop.M_rows @ e)
        rho = np.linalg.norm(e_new[act]) / np.linalg.norm(e[act])
        e = e_new / np.linalg.norm(e_new[act])
    assert rho < 0.5


def test_half_transfers_commute_with_the_mirror_extension(half_small):
    """The half-cavity transfers are the full ones on symmetric fields:
    Q_f P_h x_c = P Q_c x_c and Q_c R_h r_f = (P^T / 8) Q_f r_f, i.e. the
    full prolongation and restriction map mirror-symmetric fields to
    mirror-symmetric fields (normal components even, tangential odd)."""
    from oracle import multigrid as omg
    fr, vc = half_small
    ef, ec = vc.exts[0], vc.exts[1]
    Lf, Lc = vc.levels[0], vc.levels[1]
    Pfull = omg.prolongation(ef.gf, ec.gf, Lf.op.full.a > 0, Lc.op.full.a > 0, Lc.op.full.a)
    rng = np.random.default_rng(4)
    xc = rng.standard_normal(ec.gh.n_faces) * (Lc.op.a > 0)
    lhs = ef.Q @ (vc.P[0] @ xc)
    rhs = Pfull @ (ec.Q @ xc)
    assert np.max(abs(lhs - rhs)) <= 1e-14 * np.max(abs(rhs))
    rf = rng.standard_normal(ef.gh.n_faces) * (Lf.op.a > 0)
    lhs = ec.Q @ (vc.Rt[0] @ rf)
    rhs = (Pfull.T / 8.0) @ (ef.Q @ rf)
    assert np.max(abs(lhs - rhs)) <= 1e-14 * np.max(abs(rhs))


def test_half_vcycle_without_planes_is_the_vcycle(full_small):
    """With no PMC axis the mirror extension is the identity and the half
    V-cycle is the full one (pinned in test_oracle_multigrid)."""
    from oracle import multigrid as omg
    g, n, fr = full_small
    vc_h = sym.HalfVCycle(fr, n, H, 2.0, (), 3)
    vc_f = omg.VCycle(fr, n, H, 2.0, 3)
    act = vc_f.levels[0].op.act
    f = np.zeros(vc_f.levels[0].op.grid.n_faces)
    f[act] = np.random.default_rng(5).standard_normal(act.size)
    assert np.max(abs(vc_h(f) - vc_f(f))) <= 1e-13 * np.max(abs(vc_f(f)))


def test_symmetric_pencil_eigs_match_dense(half_small, full_small):
    """The symmetric pencil in augmented form (used for the 9-cell quarter's
    stored eigenvalues), by block Lanczos with the half V-cycle as the CG
    preconditioner, equals the dense symmetric pencil."""
    g, n, fr = full_small
    _, vc = half_small
    ext = sym.MirrorExtension((8, 8, 24), H, (0, 1))
    hop = sym.HalfOperators(ext, fr, 2.0)
    pen = sym.SymmetricPencil(hop)
    pre = sym.half_vcycle_preconditioner(vc, pen)
    lam, B, info = eigs.augmented_eigs(pen, 6, sigma_o=2.0, block=3, tol=1e-11, cg_tol=1e-12, precond=pre)
    w_ref, _ = sym.sym_dense_eigs(hop, 6)
    assert np.max(abs(lam - w_ref) / w_ref) <= 1e-10
