"""Pin of the oracle's field sampling with a closed-form mode of the PEC
unit cube: the lowest eigenvalue of the N^3 Yee cube is threefold (one mode
per axis); in the combination whose e has no x and y components, C^T b / k
on the z-edges is sin(pi i / N) sin(pi j / N) up to a constant, and the
trilinear interpolation at a point midway between two z-edges is their
mean."""
import math

import numpy as np

from oracle import eigs, fields, geometry as geo, operators as ops


def test_cube_mode_field():
    n, h = (6, 6, 6), 1.0 / 6
    op = ops.build(geo.fractions(geo.Box(), n, h), n, h, 0.0)
    lam, V = eigs.dense_eigs(op, 3)
    # the lowest eigenvalue, 2 (2 sin(pi/12) / h)^2, is threefold
    full = np.stack([op.full_face(V[:, c]) for c in range(3)], axis=1)
    exy = []
    for c in range(3):
        ex, ey, ez = fields.edge_field(op, full[:, c], lam[0])
        exy.append(np.concatenate([ex.ravel(), ey.ravel()]))
    # combination with e_x = e_y = 0
    M = np.stack(exy, axis=1)
    _, _, vt = np.linalg.svd(M)
    coef = vt[-1]
    b = full @ coef
    ex, ey, ez = fields.edge_field(op, b, lam[0])
    assert np.max(abs(ex)) + np.max(abs(ey)) <= 1e-10 * np.max(abs(ez))
    i = np.arange(n[0] + 1)
    want = np.outer(np.sin(math.pi * i / n[1]), np.sin(math.pi * i / n[0]))   # [j, i]
    got = ez[2] / ez[2][3, 3]
    assert np.max(abs(got - want)) <= 1e-10
    # interpolation at the midpoint between two z-edges along x
    p = np.array([[2.5 * h, 3 * h, 2.5 * h]])
    val = fields.sample_e(op, b, lam[0], p)[0]
    assert abs(val[2] - 0.5 * (ez[2][3, 2] + ez[2][3, 3])) <= 1e-12 * abs(val[2])
