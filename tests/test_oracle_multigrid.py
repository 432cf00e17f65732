"""Pins of the oracle V-cycle definition.

The paper's multigrid (Sec. 6) is algebraic; this project's geometric V-cycle
is a reading.  What mathematics fixes about it, and is checked here: the
V-cycle operator is symmetric (reverse smoothing order, R = P^T / 8), a
one-level cycle is the exact inverse, it contracts the error at an SPD shift,
and the coarse fractions obtained by summation are the geometric fractions
of the coarse grid.
"""
import numpy as np
import pytest

from oracle import geometry as geo, multigrid as mg


@pytest.fixture(scope="module")
def sphere16_frac():
    n, h = (16, 16, 16), 1.0 / 16
    return geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h), n, h


@pytest.mark.parametrize("sigma", [5.0, 36.0])
def test_vcycle_is_symmetric(sphere16_frac, sigma):
    fr, n, h = sphere16_frac
    vc = mg.VCycle(fr, n, h, sigma, 3)
    rng = np.random.default_rng(1)
    m = vc.levels[0].op.act.size
    u, v = rng.standard_normal(m), rng.standard_normal(m)
    lhs, rhs = u @ vc.apply_active(v), v @ vc.apply_active(u)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_one_level_is_exact_inverse(sphere16_frac):
    fr, n, h = mg.coarsen_fractions(sphere16_frac[0]), (8, 8, 8), 1.0 / 8
    vc = mg.VCycle(fr, n, h, 5.0, 1)
    op = vc.levels[0].op
    f = np.random.default_rng(2).standard_normal(op.act.size)
    x = vc.apply_active(f)
    assert np.linalg.norm(op.M_a @ x - f) < 1e-12 * np.linalg.norm(f)


def test_vcycle_contracts(sphere16_frac):
    """Stationary iteration x += B (f - M x) at sigma = 5 (SPD): the residual
    falls by at least 3x per cycle (the paper's AMG rates were 0.21-0.27)."""
    fr, n, h = sphere16_frac
    vc = mg.VCycle(fr, n, h, 5.0, 3)
    op = vc.levels[0].op
    f = np.random.default_rng(3).standard_normal(op.act.size)
    x = np.zeros_like(f)
    r0 = np.linalg.norm(f)
    for _ in range(6):
        x += vc.apply_active(f - op.M_a @ x)
    rate = (np.linalg.norm(f - op.M_a @ x) / r0) ** (1 / 6)
    assert rate < 0.33


def test_coarse_fractions_are_geometric(sphere16_frac):
    _, n, h = sphere16_frac
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h, drop_empty=False)
    coarse = mg.coarsen_fractions(fr)
    direct = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), (8, 8, 8), 2 * h, drop_empty=False)
    for s in coarse:
        assert np.max(abs(coarse[s] - direct[s])) < 1e-13


def generic_vcycle(levels_M, classes, P, coarse_sel, f, nu=2):
    """A plain V-cycle for given level matrices: Gauss--Seidel over the given
    classes (reversed on the way up), restriction P^T / 8, dense coarsest
    solve -- written out again for the tilde check below."""
    def cycle(lev, f):
        M = levels_M[lev]
        x = np.zeros_like(f)
        if lev == len(levels_M) - 1:
            s = coarse_sel
            x[s] = np.linalg.solve(M[s][:, s].toarray(), f[s])
            return x
        d = M.diagonal()
        order = classes[lev]
        for _ in range(nu):
            for ids in order:
                x[ids] += (f[ids] - M[ids] @ x) / d[ids]
        r = f - M @ x
        x += P[lev] @ cycle(lev + 1, (P[lev].T @ r) / 8.0)
        for _ in range(nu):
            for ids in order[::-1]:
                x[ids] += (f[ids] - M[ids] @ x) / d[ids]
        return x
    return cycle(0, f)


def test_tilde_vcycle_is_the_vcycle_of_the_scaled_operator(sphere16_frac):
    """Sec. 5.3, eq. fullMat2: the tilde V-cycle (transfers conjugated by
    A^1/2) equals A^-1/2 B~ A^-1/2, where B~ is the plain V-cycle built on
    the scaled matrices M~ = A^-1/2 M A^-1/2 of every level with the
    unscaled transfers P -- constructed independently here."""
    import scipy.sparse as sp
    fr, n, h = sphere16_frac
    vt = mg.VCycle(fr, n, h, 5.0, 3, tilde=True)
    vp = mg.VCycle(fr, n, h, 5.0, 3)
    Ms, cls, inv_sqrt = [], [], []
    for L in vp.levels:
        s = np.where(L.active, 1.0 / np.sqrt(np.where(L.active, L.op.a, 1.0)), 0.0)
        inv_sqrt.append(s)
        Ms.append((sp.diags(s) @ L.M @ sp.diags(s)).tocsr())
        cls.append([L.classes[c] for c in vp.ORDER])
    rng = np.random.default_rng(3)
    f = np.zeros(vp.levels[0].op.grid.n_faces)
    act = vp.levels[0].op.act
    f[act] = rng.standard_normal(act.size)
    ref = inv_sqrt[0] * generic_vcycle(Ms, cls, vp.P, vp.coarse_sel, inv_sqrt[0] * f)
    got = vt(f)
    assert np.max(abs(got - ref)) <= 1e-12 * np.max(abs(ref))
    # symmetric, and a different preconditioner from the method's
    u = rng.standard_normal(act.size)
    lhs, rhs = u @ vt.apply_active(f[act]), f[act] @ vt.apply_active(u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.max(abs(got - vp(f))) > 1e-3 * np.max(abs(got))
