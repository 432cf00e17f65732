"""GPU parity: every HIP building block against the oracle, element by element.

The library is built from the oracle's own fractions (user geometry), so the
comparison isolates the kernels.  Grids: the 16^3 node-centred sphere
(R = 0.45, the small configuration) and a ragged 12 x 10 x 14 grid with an
off-centre ellipsoid (partial blocks, non-cubic strides).

Tolerances (norm-wise, ||y_gpu - y_ref||_inf / ||y_ref||_inf):
  FP64 kernels 1e-12 (the stencil-apply bar); FP32 kernels 2e-5 (FP32 unit
  roundoff 6e-8 times the ~15-term stencil sums and a few ulps of the
  1/h^2 scaling); iterative results (projection, solves) 1e-9.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import geometry as geo, multigrid as omg, operators as ops
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "sphere16": dict(n=(16, 16, 16), h=1.0 / 16, geom=geo.sphere((0.5, 0.5, 0.5), 0.45),
                     sigma=5.0, levels=3),
    "ragged": dict(n=(12, 10, 14), h=1.0 / 14, geom=geo.Ellipsoid((0.45, 0.36, 0.5), (0.38, 0.31, 0.42)),
                   sigma=3.0, levels=2),
}


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_1301_3794_amd import dm
    c = CASES[request.param]
    n, h = c["n"], c["h"]
    fr = geo.fractions(c["geom"], n, h)
    oop = ops.build(fr, n, h, c["sigma"])
    vc = omg.VCycle(fr, n, h, c["sigma"], c["levels"])
    fr7 = lay.fractions_to_padded(fr, n)
    op = dm.Operator(dm.user_fractions(fr7), n, h, c["sigma"], levels=c["levels"])
    print(f"[case] {request.param} n={n} levels={c['levels']}", flush=True)
    yield dict(c, name=request.param, fr=fr, oop=oop, vc=vc, op=op, dm=dm)
    op.close()


def dev(x, dtype=None):
    return torch.tensor(x, dtype=dtype or torch.float64, device="cuda")


def full_random(oop, seed):
    x = np.zeros(oop.grid.n_faces)
    x[oop.act] = np.random.default_rng(seed).standard_normal(oop.act.size)
    return x


def test_layout_matches(case):
    lay0 = case["op"].layout(0)
    assert lay0["active_faces"] == case["oop"].act.size
    assert lay0["active_cells"] == case["oop"].cact.size
    assert lay0["levels"] == case["levels"]


@pytest.mark.parametrize("which", ["M", "K", "A"])
def test_apply_fp64(case, which):
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    x = full_random(oop, 1)
    y = op.apply({"M": dm.APPLY_M, "K": dm.APPLY_K, "A": dm.APPLY_A}[which],
                 dev(lay.faces_to_padded(x, n)), op.face_tensor())
    ref = {"M": oop.M, "K": oop.K, "A": oop.A}[which] @ x
    got = lay.faces_from_padded(y.cpu().numpy(), n)
    assert rel_inf(got, ref) <= 1e-12
    # padding and inactive faces stay exactly zero
    yp = y.cpu().numpy()
    assert np.all(yp[lay.faces_to_padded(np.ones(oop.grid.n_faces), n) == 0] == 0)


def test_apply_fp32(case):
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    x = full_random(oop, 2)
    y = op.apply(dm.APPLY_M, dev(lay.faces_to_padded(x, n), torch.float32),
                 op.face_tensor(dtype=torch.float32))
    ref = oop.M @ x
    assert rel_inf(lay.faces_from_padded(y.double().cpu().numpy(), n), ref) <= 2e-5


def test_scalar_operators(case):
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    x = full_random(oop, 3)
    g = op.apply(dm.APPLY_DA, dev(lay.faces_to_padded(x, n)), op.cell_tensor())
    ref = oop.D @ (oop.a * x)
    assert rel_inf(lay.cells_from_padded(g.cpu().numpy(), n), ref) <= 1e-12
    psi = np.zeros(oop.grid.n_cells)
    psi[oop.cact] = np.random.default_rng(4).standard_normal(oop.cact.size)
    y = op.apply(dm.APPLY_DT, dev(lay.cells_to_padded(psi, n)), op.face_tensor())
    ref = np.zeros(oop.grid.n_faces)
    ref[oop.act] = oop.D_a.T @ psi[oop.cact]
    assert rel_inf(lay.faces_from_padded(y.cpu().numpy(), n), ref) <= 1e-12
    s = op.apply(dm.APPLY_S, dev(lay.cells_to_padded(psi, n)), op.cell_tensor())
    ref = np.zeros(oop.grid.n_cells)
    ref[oop.cact] = oop.S_a @ psi[oop.cact]
    assert rel_inf(lay.cells_from_padded(s.cpu().numpy(), n), ref) <= 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_residual(case, prec):
    op, oop, n = case["op"], case["oop"], case["n"]
    dt = torch.float64 if prec == 64 else torch.float32
    x, f = full_random(oop, 5), full_random(oop, 6)
    r = op.residual(dev(lay.faces_to_padded(f, n), dt), dev(lay.faces_to_padded(x, n), dt),
                    op.face_tensor(dtype=dt))
    ref = f - oop.M @ x
    tol = 1e-12 if prec == 64 else 2e-5
    assert rel_inf(lay.faces_from_padded(r.double().cpu().numpy(), n), ref) <= tol


@pytest.mark.parametrize("reverse", [False, True])
def test_smoother_sweep(case, reverse):
    op, vc, n = case["op"], case["vc"], case["n"]
    L = vc.levels[0]
    x0, f = full_random(L.op, 7), full_random(L.op, 8)
    xg = dev(lay.faces_to_padded(x0, n))
    op.smooth(dev(lay.faces_to_padded(f, n)), xg, sweeps=2, reverse=reverse)
    ref = x0.copy()
    order = vc.ORDER[::-1] if reverse else vc.ORDER
    for _ in range(2):
        vc._smooth(L, ref, f, order)
    assert rel_inf(lay.faces_from_padded(xg.cpu().numpy(), n), ref) <= 1e-12


def test_transfers(case):
    op, vc, n = case["op"], case["vc"], case["n"]
    nc = tuple(x // 2 for x in n)
    Lf, Lc = vc.levels[0], vc.levels[1]
    r = full_random(Lf.op, 9)
    fc = op.restrict(dev(lay.faces_to_padded(r, n)), op.face_tensor(level=1))
    ref = vc.P[0].T @ r / 8.0
    assert rel_inf(lay.faces_from_padded(fc.cpu().numpy(), nc), ref) <= 1e-12
    xc = full_random(Lc.op, 10)
    x0 = full_random(Lf.op, 11)
    xg = dev(lay.faces_to_padded(x0, n))
    op.prolong_add(dev(lay.faces_to_padded(xc, nc)), xg)
    ref = x0 + vc.P[0] @ xc
    assert rel_inf(lay.faces_from_padded(xg.cpu().numpy(), n), ref) <= 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_vcycle(case, prec):
    op, vc, n = case["op"], case["vc"], case["n"]
    dt = torch.float64 if prec == 64 else torch.float32
    f = full_random(vc.levels[0].op, 12)
    x = op.vcycle(dev(lay.faces_to_padded(f, n), dt), op.face_tensor(dtype=dt))
    ref = vc(f)
    tol = 1e-12 if prec == 64 else 5e-5
    assert rel_inf(lay.faces_from_padded(x.double().cpu().numpy(), n), ref) <= tol


def test_projection(case):
    from oracle import eigs as oeigs
    op, oop, n = case["op"], case["oop"], case["n"]
    b = full_random(oop, 13)
    out = op.project(dev(lay.faces_to_padded(b, n)), op.face_tensor(), rtol=1e-13)
    ref = np.zeros_like(b)
    ref[oop.act] = oeigs.Projector(oop, tol=1e-13)(b[oop.act])
    got = lay.faces_from_padded(out.cpu().numpy(), n)
    assert rel_inf(got, ref) <= 1e-9
    # divergence-free to rounding: D A (P b) = 0
    div = oop.D @ (oop.a * got)
    assert np.max(abs(div)) <= 1e-9 * np.max(abs(oop.D @ (oop.a * b)))


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32", "pcg64"])
def test_solve(case, mode):
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    m = {"fgmres64": dm.SOLVE_FGMRES_MG64, "fgmres32": dm.SOLVE_FGMRES_MG32, "pcg64": dm.SOLVE_PCG64}[mode]
    f = full_random(oop, 14)
    x = op.face_tensor()
    info = op.solve(dev(lay.faces_to_padded(f, n)), x, mode=m, rtol=1e-11, maxit=200)
    assert info["status"] == 0, info
    ref = np.zeros_like(f)
    ref[oop.act] = sla.spsolve(oop.M_a.tocsc(), f[oop.act])
    assert rel_inf(lay.faces_from_padded(x.cpu().numpy(), n), ref) <= 1e-9
    assert info["rel_residual"] <= 1e-11


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32"])
def test_solve_reads_only_lines_with_active_faces(case, mode):
    """The FGMRES reductions, updates and preconditioner casts visit only the
    128-byte lines (16 doubles) of a face vector that hold an active face:
    values of f in the other lines change nothing, and x stays zero there."""
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    m = dm.SOLVE_FGMRES_MG64 if mode == "fgmres64" else dm.SOLVE_FGMRES_MG32
    active = np.asarray(op.fractions(0))[:3].reshape(-1) != 0.0
    nline = (active.size + 15) // 16
    padded = np.zeros(nline * 16, dtype=bool)
    padded[:active.size] = active
    empty = np.flatnonzero(~padded.reshape(nline, 16).any(axis=1))
    assert empty.size > 0
    f = lay.faces_to_padded(full_random(oop, 16), n)
    junk = f.copy()
    for line in empty[:: max(1, empty.size // 40)]:
        junk[line * 16:min(active.size, line * 16 + 16)] = 1e3
    x1, x2 = op.face_tensor(), op.face_tensor()
    i1 = op.solve(dev(f), x1, mode=m, rtol=1e-11, maxit=200)
    i2 = op.solve(dev(junk), x2, mode=m, rtol=1e-11, maxit=200)
    assert i1["status"] == 0 and i2["status"] == 0
    assert i1["iterations"] == i2["iterations"]
    a, b = x1.cpu().numpy(), x2.cpu().numpy()
    assert np.array_equal(a, b)
    outside = np.repeat(~padded.reshape(nline, 16).any(axis=1), 16)[:active.size]
    assert np.all(b[outside] == 0.0)
