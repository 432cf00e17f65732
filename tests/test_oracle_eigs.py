"""Pins of the oracle eigensolvers (Sec. 4.1, eqs. shiftInv / fullMat; Sec. 6.2).

References: the closed-form Yee spectrum of the PEC cube, dense eigh on small
grids, the analytic TM modes of the spherical cavity (roots of
[x j_l(x)]' = 0) with second-order convergence, and the algebraic
properties of the projection (eq. proj, P^2 = P, gradients removed).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import optimize, special

from oracle import eigs, geometry as geo, operators as ops


def tm_root(l, lo, hi):
    """Root of d/dx [x j_l(x)] = j_l(x) + x j_l'(x) (TM modes of a PEC sphere)."""
    f = lambda x: special.spherical_jn(l, x) + x * special.spherical_jn(l, x, derivative=True)  # noqa: E731
    return optimize.brentq(f, lo, hi, xtol=1e-15)


def test_box_lanczos_matches_closed_form():
    N = 8
    h = 1.0 / N
    fr = geo.fractions(geo.Box(), (N, N, N), h)
    op = ops.build(fr, (N, N, N), h, 5.0)
    lam, B, info = eigs.lanczos_eigs(op, 5, sigma_o=5.0, block=4, tol=1e-11)
    ref = sorted(sum((2 * math.sin(math.pi * x / (2 * N)) / h) ** 2 for x in m)
                 for m in itertools.product(range(3), repeat=3) if sum(x > 0 for x in m) >= 2)
    # (1,1,0)x3 then (1,1,1)x2: 2 (16 sin(pi/16))^2 (x3), 3 (16 sin(pi/16))^2 (x2)
    want = [ref[0]] * 3 + [ref[3]] * 2
    assert want[0] == pytest.approx(19.4868396771, abs=1e-9)
    assert want[3] == pytest.approx(29.2302595157, abs=1e-9)
    assert np.max(abs(lam - want) / np.array(want)) < 1e-10
    assert info["residuals"].max() <= 1e-11


def test_dense_vs_lanczos_sphere_8():
    n, h = (8, 8, 8), 1.0 / 8
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    op = ops.build(fr, n, h, 5.0)
    w, V = eigs.dense_eigs(op, 6)
    lam, B, info = eigs.lanczos_eigs(op, 6, sigma_o=5.0, block=4, tol=1e-11)
    assert np.max(abs(lam - w) / w) < 1e-12
    for c in range(6):
        assert eigs.eig_residual(op, w[c], V[:, c]) < 1e-12
        assert eigs.eig_residual(op, lam[c], B[:, c]) < 1e-11
        assert eigs.div_residual(op, B[:, c]) < 1e-10
    # A-orthonormal Ritz vectors
    G = B.T @ (op.a_a[:, None] * B)
    assert np.max(abs(G - np.eye(6))) < 1e-12


def test_augmented_route_matches_dense_sphere_8():
    """Sec. 5.1: the EM pairs of (K + G, A), selected by zero divergence, are
    the nonzero pairs of (K, A)."""
    n, h = (8, 8, 8), 1.0 / 8
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    op = ops.build(fr, n, h, 5.0)
    w, _ = eigs.dense_eigs(op, 6)
    lam, B, info = eigs.augmented_eigs(op, 6, sigma_o=5.0, block=4, tol=1e-11)
    assert np.max(abs(lam - w) / w) < 1e-12
    assert info["residuals"].max() <= 1e-11


def test_sphere_tm11_second_order_convergence():
    """Sec. 6.2 / Fig. fig:freqErr3d: with every cut face kept the
    Dey--Mittra frequencies converge at second order.  TM_11 of a sphere of
    radius R = 0.45: k = x_11 / R, x_11 the first root of [x j_1(x)]' = 0.
    The triplet is exactly degenerate on a node-centred grid (O_h)."""
    x11 = tm_root(1, 2.0, 3.5)
    assert x11 == pytest.approx(2.743707, abs=1e-6)
    k2 = (x11 / 0.45) ** 2
    errs = []
    ns = (8, 12, 16, 20)
    for N in ns:
        h = 1.0 / N
        fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), (N, N, N), h)
        op = ops.build(fr, (N, N, N), h, 15.0)
        lam, _, _ = eigs.lanczos_eigs(op, 3, sigma_o=15.0, block=3, tol=1e-9)
        assert (lam.max() - lam.min()) / lam.min() < 1e-12
        errs.append(abs(lam[0] - k2) / k2)
    p = np.polyfit(np.log(1.0 / np.array(ns)), np.log(errs), 1)[0]
    assert 1.6 <= p <= 2.4
    assert errs[-1] < 4.5e-3


def test_projection_properties(sphere16):
    """eq. proj: P_DM is a projection (P^2 = P), its range is divergence-free
    (D A P b = 0), it removes gradients (P D^T psi = 0) and keeps the curl
    part A^-1 C L e of the Helmholtz decomposition."""
    fr, op = sphere16
    P = eigs.Projector(op, tol=1e-14)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(op.act.size)
    pb = P(b)
    scale = np.linalg.norm(op.D_a @ (op.a_a * b))
    assert np.linalg.norm(op.D_a @ (op.a_a * pb)) < 1e-11 * scale
    assert np.linalg.norm(P(pb) - pb) < 1e-11 * np.linalg.norm(pb)
    psi = rng.standard_normal(op.cact.size)
    grad = op.D_a.T @ psi
    assert np.linalg.norm(P(grad)) < 1e-10 * np.linalg.norm(grad)
    # curl part: b = A^-1 C L e for a random edge field e
    e = rng.standard_normal(op.grid.n_edges)
    curl = (op.Ct.T @ (op.l * e))[op.act] / op.a_a
    assert np.linalg.norm(P(curl) - curl) < 1e-10 * np.linalg.norm(curl)


def test_eig_residual_definition():
    """rho = ||K b - lam A b||_{A^-1} / (lam ||b||_A) is scale invariant and
    zero for exact eigenpairs; a wrong lambda gives |dlam| / lam."""
    n, h = (6, 6, 6), 1.0 / 6
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    op = ops.build(fr, n, h, 0.0)
    w, V = eigs.dense_eigs(op, 2)
    assert eigs.eig_residual(op, w[0], 3.7 * V[:, 0]) < 1e-12
    assert eigs.eig_residual(op, w[0] * (1 + 1e-6), V[:, 0]) == pytest.approx(1e-6 / (1 + 1e-6), rel=1e-6)


def test_div_residual_known_values():
    """||V^-1/2 D A b|| / ||b||_A (Sec. 5.1) on the PEC box, where a = v = 1:
    for b = D^T psi with psi a Neumann eigenvector of the cell Laplacian,
    psi = prod cos(pi m_a (i_a + 1/2) / N), D D^T psi = mu psi with
    mu = sum (2 sin(pi m_a / 2N) / h)^2, so the value is sqrt(mu); for a
    curl b = C e it is zero (D C = 0)."""
    n, h = (6, 5, 4), 0.2
    fr = geo.fractions(geo.Box(), n, h)
    op = ops.build(fr, n, h, 0.0)
    g = op.grid
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for m in ((1, 0, 0), (0, 2, 1), (3, 1, 2)):
        psi = (np.cos(math.pi * m[0] * (i + 0.5) / n[0]) * np.cos(math.pi * m[1] * (j + 0.5) / n[1])
               * np.cos(math.pi * m[2] * (k + 0.5) / n[2])).ravel()
        mu = sum((2.0 * math.sin(math.pi * m[a] / (2 * n[a])) / h) ** 2 for a in range(3))
        b = (op.D.T @ psi)[op.act]
        assert eigs.div_residual(op, b) == pytest.approx(math.sqrt(mu), rel=1e-12)
    # tangential e vanishes on the conducting walls (l = 0 there)
    e = np.random.default_rng(0).standard_normal(g.n_edges) * (op.l > 0)
    b = (op.Ct.T @ e)[op.act]
    assert eigs.div_residual(op, b) <= 1e-13 / h
