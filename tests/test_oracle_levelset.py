"""Pins of the tetrahedral cut fractions of a sampled level set (Sec. 6.1:
cut-cell volumes from tetrahedral subvolumes conforming to the surface).

* A planar surface is represented exactly by the piecewise-linear
  interpolant, so every fraction equals the closed form of the half-space
  x + y < c: edges and faces are intervals and triangles/trapezoids of the
  unit square, cells their prisms.
* A sphere: the volume and every interior plane's area sum converge to
  4 pi R^3 / 3 and pi rho^2 at second order in h / s.
* The library's fractions (its own case formulas: corner simplices and a
  prism cut into three tetrahedra) equal the oracle's (convex hulls by
  Qhull) on a ragged off-centre ellipsoid, refinements 1 to 3.
"""
import math

import numpy as np
import pytest

from oracle import geometry as geo
import layout as lay


def half_plane_area(t):
    """Area of {(x, y) in [0, 1]^2 : x + y < t}."""
    if t <= 0.0:
        return 0.0
    if t <= 1.0:
        return 0.5 * t * t
    if t < 2.0:
        return 1.0 - 0.5 * (2.0 - t) ** 2
    return 1.0


@pytest.mark.parametrize("s", [1, 2])
def test_plane_is_exact(s):
    n, h, c = (5, 4, 3), 1.0, 3.37
    phi = geo.sample_levelset(lambda x, y, z: x + y - c, n, h, s)
    fr = geo.levelset_fractions(phi, s, n, drop_empty=False)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                assert fr["v"][k, j, i] == pytest.approx(half_plane_area(c - i - j), abs=1e-12)
                assert fr["az"][k, j, i] == (0.0 if k == 0 else pytest.approx(half_plane_area(c - i - j), abs=1e-12))
    # x-face at x = i: {y in [j, j+1] : i + y < c}; x-edge at (j, k): {x in [i, i+1] : x + j < c}
    for j in range(n[1]):
        for i in range(1, n[0]):
            want = min(1.0, max(0.0, c - i - j))
            assert fr["ax"][1, j, i] == pytest.approx(want, abs=1e-12)
    for j in range(1, n[1]):
        for i in range(n[0]):
            want = min(1.0, max(0.0, c - i - j))
            assert fr["lx"][1, j, i] == pytest.approx(want, abs=1e-12)


def test_sphere_converges_at_second_order():
    n, h, R = (8, 8, 8), 1.0 / 8, 0.45
    exact_v = 4.0 / 3.0 * math.pi * R ** 3
    k_plane = 4
    rho2 = R * R - (k_plane * h - 0.5) ** 2
    verr, aerr = [], []
    for s in (1, 2, 4):
        phi = geo.sample_levelset(lambda x, y, z: np.sqrt((x - .5) ** 2 + (y - .5) ** 2 + (z - .5) ** 2) - R, n, h, s)
        fr = geo.levelset_fractions(phi, s, n)
        verr.append(abs(fr["v"].sum() * h ** 3 - exact_v))
        aerr.append(abs(fr["az"][k_plane].sum() * h * h - math.pi * rho2))
    assert verr[1] < verr[0] / 3 and verr[2] < verr[1] / 3
    assert aerr[1] < aerr[0] / 3 and aerr[2] < aerr[1] / 3


def test_library_matches_oracle():
    from paper_1301_3794_amd import dm
    n, h = (9, 7, 8), 1.0 / 8

    def f(x, y, z):
        return ((x - 0.56) / 0.49) ** 2 + ((y - 0.44) / 0.37) ** 2 + ((z - 0.5) / 0.45) ** 2 - 1.0
    for s in (1, 2, 3):
        phi = geo.sample_levelset(f, n, h, s)
        ref = lay.fractions_to_padded(geo.levelset_fractions(phi, s, n), n)
        got = dm.compute_fractions(dm.levelset(phi, s), n, h)
        assert np.max(abs(got - ref)) <= 1e-13, s
