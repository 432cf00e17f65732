"""Pins of the oracle's cut fractions (Sec. 2 and Sec. 5.1 definitions).

Checked against what geometry fixes independently of the oracle's formulas:
measure sums, direct 2-D / nested quadrature of the indicator, symmetry,
and the numbers printed with the paper's sphere benchmark.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import geometry as geo


@pytest.mark.parametrize("rho,rect", [
    (1.0, (-2.0, 2.0, -2.0, 2.0)),       # rectangle holds the whole disk
    (0.3, (0.0, 1.0, 0.0, 1.0)),         # corner at the centre: quarter disk
    (1.0, (-0.2, 0.3, -0.1, 0.4)),       # rectangle inside the disk
    (1.0, (1.0, 2.0, 0.0, 1.0)),         # touches along a point only
])
def test_disk_rect_area_special_cases(rho, rect):
    y0, y1, z0, z1 = rect
    exact = {0: math.pi * rho * rho, 1: math.pi * rho * rho / 4,
             2: (y1 - y0) * (z1 - z0), 3: 0.0}
    case = [(-2.0, 2.0, -2.0, 2.0), (0.0, 1.0, 0.0, 1.0),
            (-0.2, 0.3, -0.1, 0.4), (1.0, 2.0, 0.0, 1.0)].index(rect)
    assert geo.disk_rect_area(rho, *rect) == pytest.approx(exact[case], abs=1e-15)


def test_disk_rect_area_vs_2d_quadrature():
    """Closed-form chord integral vs SciPy 2-D quadrature of the indicator."""
    rng = np.random.default_rng(7)
    for _ in range(25):
        rho = rng.uniform(0.2, 1.0)
        y0, z0 = rng.uniform(-1.1, 0.9, size=2)
        y1, z1 = y0 + rng.uniform(0.01, 0.5), z0 + rng.uniform(0.01, 0.5)

        def lo(y):
            s = math.sqrt(max(rho * rho - y * y, 0.0))
            return min(max(z0, -s), z1)

        def hi(y):
            s = math.sqrt(max(rho * rho - y * y, 0.0))
            return max(min(z1, s), lo(y))

        ref, _ = integrate.dblquad(lambda z, y: 1.0, y0, y1, lo, hi, epsabs=1e-14, epsrel=1e-12)
        assert geo.disk_rect_area(rho, y0, y1, z0, z1) == pytest.approx(ref, abs=1e-11)


def test_sphere_measure_sums(sphere16):
    fr, _ = sphere16
    n, h, R, c = 16, 1.0 / 16, 0.45, 0.5
    # volume: sum of v h^3 is the ball volume
    assert fr["v"].sum() * h ** 3 == pytest.approx(4 * math.pi * R ** 3 / 3, rel=1e-13)
    # every x = ih plane: sum of a h^2 is the disk area of the section
    for i in range(1, n):
        rho2 = R * R - (i * h - c) ** 2
        want = math.pi * rho2 if rho2 > 0 else 0.0
        assert fr["ax"][:, :, i].sum() * h * h == pytest.approx(want, abs=1e-14)
        assert fr["ay"][:, i, :].sum() * h * h == pytest.approx(want, abs=1e-14)
        assert fr["az"][i, :, :].sum() * h * h == pytest.approx(want, abs=1e-14)
    # every x-line (y = jh, z = kh): sum of l h is the chord
    for j in range(1, n):
        for k in range(1, n):
            d2 = (j * h - c) ** 2 + (k * h - c) ** 2
            want = 2 * math.sqrt(R * R - d2) if d2 < R * R else 0.0
            assert fr["lx"][k, j, :].sum() * h == pytest.approx(want, abs=1e-14)


def test_ellipsoid_measure_sums():
    cen, semi = (0.52, 0.47, 0.5), (0.41, 0.33, 0.27)
    n, h = (12, 12, 12), 1.0 / 12
    fr = geo.fractions(geo.Ellipsoid(cen, semi), n, h, drop_empty=False)
    vol = 4 * math.pi * semi[0] * semi[1] * semi[2] / 3
    assert fr["v"].sum() * h ** 3 == pytest.approx(vol, rel=1e-12)
    for i in range(1, 12):
        t = 1 - ((i * h - cen[0]) / semi[0]) ** 2
        want = math.pi * semi[1] * semi[2] * t if t > 0 else 0.0
        assert fr["ax"][:, :, i].sum() * h * h == pytest.approx(want, abs=1e-14)
        t = 1 - ((i * h - cen[2]) / semi[2]) ** 2
        want = math.pi * semi[0] * semi[1] * t if t > 0 else 0.0
        assert fr["az"][i, :, :].sum() * h * h == pytest.approx(want, abs=1e-14)


def test_cut_cell_volume_vs_nested_quadrature(sphere16):
    """v of cut cells vs nested quadrature of the z-chord length over the
    cell's x-y square (independent of the disk/rectangle closed form).  The
    inner y-integral is split where the chord function of y has kinks: where
    the line leaves the ball, or its chord end crosses z0 or z0 + h."""
    fr, _ = sphere16
    h, R, c = 1.0 / 16, 0.45, 0.5
    cut = np.argwhere((fr["v"] > 0) & (fr["v"] < 1))
    rng = np.random.default_rng(3)
    for k, j, i in cut[rng.choice(len(cut), 6, replace=False)]:
        x0, y0, z0 = i * h, j * h, k * h

        def chord(y, x):
            d2 = (x - c) ** 2 + (y - c) ** 2
            if d2 >= R * R:
                return 0.0
            s = math.sqrt(R * R - d2)
            return geo.interval_overlap(z0, z0 + h, c - s, c + s)

        def inner(x):
            pts = []
            for zz in (None, z0, z0 + h):
                r2 = R * R - (x - c) ** 2 - (0.0 if zz is None else (zz - c) ** 2)
                if r2 > 0:
                    pts += [c - math.sqrt(r2), c + math.sqrt(r2)]
            pts = sorted(p for p in pts if y0 < p < y0 + h)
            val, _ = integrate.quad(chord, y0, y0 + h, args=(x,), points=pts or None,
                                    epsabs=1e-16, epsrel=1e-13, limit=200)
            return val

        ref, _ = integrate.quad(inner, x0, x0 + h, epsabs=1e-16, epsrel=1e-12, limit=200)
        assert fr["v"][k, j, i] == pytest.approx(ref / h ** 3, abs=1e-10)


def test_node_centred_sphere_is_octahedrally_symmetric(sphere16):
    fr, _ = sphere16
    ax, ay, az = fr["ax"], fr["ay"], fr["az"]
    # mirror x -> 1 - x maps x-face i to 16 - i and cell i to 15 - i
    assert np.max(abs(ax - ax[:, :, ::-1])) < 1e-14
    assert np.max(abs(fr["v"] - fr["v"][:, :, ::-1])) < 1e-13
    # swapping x <-> y maps ax[k, j, i] to ay[k, i, j]
    assert np.max(abs(ax - np.transpose(ay, (0, 2, 1)))) < 1e-14
    assert np.max(abs(ax - np.transpose(az, (2, 1, 0)))) < 5e-14
    assert np.max(abs(fr["v"] - np.transpose(fr["v"], (0, 2, 1)))) < 1e-13


def test_paper_sphere_component_counts():
    """Sphere of radius 0.49 L centred on a node: faces with a > 0 number
    7,224 / 53,160 / 405,876 at 16^3 / 32^3 / 64^3, the component counts of
    the first (commented-out) row of Table tab:invPerf; the PEC cube has
    3 (N - 1) N^2 = 11,520 / 95,232 / 774,144."""
    for n, sph, cube in ((16, 7224, 11520), (32, 53160, 95232), (64, 405876, 774144)):
        h = 1.0 / n
        assert geo.count_active_faces(geo.sphere((0.5, 0.5, 0.5), 0.49), (n, n, n), h) == sph
        assert geo.count_active_faces(geo.Box(), (n, n, n), h) == cube


def test_paper_smallest_area_fraction():
    """Sec. 6.1: with no face neglected the smallest area fraction met in
    the sphere runs (r = 0.49 L, 16^3..64^3) was 6e-4."""
    mins = []
    for n in (16, 32, 64):
        h = 1.0 / n
        g = geo.sphere((0.5, 0.5, 0.5), 0.49)
        a = geo.face_fractions(g, (n, n, n), h, 0)  # symmetric: x-faces suffice
        mins.append(a[a > 0].min())
    assert 5.5e-4 <= min(mins) <= 6.5e-4
    assert round(min(mins), 4) == 6e-4


def test_faces_of_empty_cells_are_dropped():
    """A face with area next to a cell of volume 0 is dropped; nothing else is."""
    v = np.ones((2, 3, 4))
    v[1, 2, 3] = 0.0
    fr = dict(v=v, ax=np.full((2, 3, 5), 0.5), ay=np.full((2, 4, 4), 0.5), az=np.full((3, 3, 4), 0.5))
    out = geo.drop_faces_of_empty_cells(fr)
    # the empty cell (i, j, k) = (3, 2, 1) owns x-faces i = 3, 4; y-faces j = 2, 3; z-faces k = 1, 2
    assert np.argwhere(out["ax"] == 0).tolist() == [[1, 2, 3], [1, 2, 4]]
    assert np.argwhere(out["ay"] == 0).tolist() == [[1, 2, 3], [1, 3, 3]]
    assert np.argwhere(out["az"] == 0).tolist() == [[1, 2, 3], [2, 2, 3]]
    assert out["v"] is fr["v"]


@pytest.mark.parametrize("body", ["sphere", "bor"])
def test_window_origin_reproduces_the_full_grid(body):
    """fractions(..., origin=o) of a window equal the full grid's fractions
    on the window's interior (its own boundary is a wall), entry for entry."""
    if body == "sphere":
        g, n, h = geo.sphere((0.5, 0.5, 0.5), 0.45), (16, 16, 16), 1.0 / 16
    else:
        g, n, h = geo.EllipticCells((0.5, 0.5), 0.03, 2, 0.4, 0.18, 0.5, 0.2), (16, 16, 20), 1.0 / 16
    o, w = (0, 5, 3), (6, 7, 8)     # a window across the cut surface
    full = geo.fractions(g, n, h, drop_empty=False)
    win = geo.fractions(g, w, h, drop_empty=False, origin=o)
    cut = 0
    for name in ("ax", "ay", "az", "lx", "ly", "lz", "v"):
        a = full[name][o[2] + 1:o[2] + w[2], o[1] + 1:o[1] + w[1], o[0] + 1:o[0] + w[0]]
        b = win[name][1:w[2], 1:w[1], 1:w[0]]
        assert np.array_equal(a, b), name
        cut += int(np.sum((a > 0) & (a < 1)))
    assert cut > 20


def test_cell_touching_a_pole_vs_chord_integral():
    """A 40^3 cell whose face x = 0.95 touches the sphere's pole: the section
    radius grows like the square root of the distance to the pole there.
    Independent value: the 2-D integral over (y, z) of the chord length in
    x inside the cell (the old adaptive integration in x was off by 5e-11)."""
    n, h = (40, 40, 40), 1.0 / 40
    g = geo.sphere((0.5, 0.5, 0.5), 0.45)
    i, j, k = 37, 20, 20
    x0, x1 = i * h, (i + 1) * h

    def chord(z, y):
        r2 = 0.45 ** 2 - (y - 0.5) ** 2 - (z - 0.5) ** 2
        if r2 <= 0.0:
            return 0.0
        s = math.sqrt(r2)
        return max(0.0, min(x1, 0.5 + s) - max(x0, 0.5 - s))

    ref, err = integrate.dblquad(chord, j * h, (j + 1) * h, k * h, (k + 1) * h, epsabs=1e-19, epsrel=1e-14)
    assert err / h ** 3 <= 1e-12
    assert geo.cell_fraction(g, n, h, i, j, k) == pytest.approx(ref / h ** 3, abs=2e-12)
