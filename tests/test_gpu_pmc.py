"""GPU parity with PMC symmetry planes (quarter cavity, Sec. 6.3).

A two-cell elliptic cavity on a 16 x 16 x 24 full grid (h = 1/16); the
library runs the quarter x, y >= 0 (8 x 8 x 24, PMC planes at x = 0 and
y = 0) from the oracle's quarter fractions.  The oracle's half-cavity
operators are the full cavity's rows on symmetric fields (oracle/symmetry.py):
apply, residual, smoother, transfers and V-cycle are compared element by
element (FP64 1e-12, FP32 2e-5 / 5e-5), and the eigenvalues with the
symmetric pencil's dense eigenvalues (1e-10).  The block projection
(whose conjugate gradients skip the cell units without an active cell or a
ghost image) matches the single-vector one to 1e-12.
"""
import numpy as np
import pytest

from oracle import geometry as geo, symmetry as sym
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = 1.0 / 16
NH = (8, 8, 24)
SIGMA = 2.0


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def case():
    from paper_1301_3794_amd import dm
    g = geo.EllipticCells((8 * H, 8 * H), 0.0, 2, 0.4, 0.18, 0.5, 0.25)
    fr_full = geo.fractions(g, (16, 16, 24), H)
    ext = sym.MirrorExtension(NH, H, (0, 1))
    hop = sym.HalfOperators(ext, fr_full, SIGMA)
    vc = sym.HalfVCycle(fr_full, NH, H, SIGMA, (0, 1), 3)
    fr7 = lay.fractions_to_padded(ext.half_fractions(fr_full), NH)
    op = dm.Operator(dm.user_fractions(fr7, bc_lo=(dm.BC_PMC, dm.BC_PMC, dm.BC_PEC)), NH, H, SIGMA,
                     levels=3)
    print("[case] quarter two-cell PMC", NH, flush=True)
    yield dict(dm=dm, hop=hop, vc=vc, op=op, ext=ext)
    op.close()


def dev(x, dtype=torch.float64):
    return torch.tensor(x, dtype=dtype, device="cuda")


def rnd(hop, seed):
    x = np.zeros(hop.grid.n_faces)
    x[hop.act] = np.random.default_rng(seed).standard_normal(hop.act.size)
    return x


def test_active_sets(case):
    lay0 = case["op"].layout(0)
    assert lay0["active_faces"] == case["hop"].act.size


@pytest.mark.parametrize("which", ["M", "K"])
def test_apply(case, which):
    dm, op, hop = case["dm"], case["op"], case["hop"]
    x = rnd(hop, 1)
    y = op.apply(dm.APPLY_M if which == "M" else dm.APPLY_K, dev(lay.faces_to_padded(x, NH)), op.face_tensor())
    ref = (hop.M_rows if which == "M" else hop.K_rows) @ x
    assert rel_inf(lay.faces_from_padded(y.cpu().numpy(), NH), ref) <= 1e-12


def test_apply_fp32_and_residual(case):
    dm, op, hop = case["dm"], case["op"], case["hop"]
    x, f = rnd(hop, 2), rnd(hop, 3)
    y = op.apply(dm.APPLY_M, dev(lay.faces_to_padded(x, NH), torch.float32), op.face_tensor(dtype=torch.float32))
    assert rel_inf(lay.faces_from_padded(y.double().cpu().numpy(), NH), hop.M_rows @ x) <= 2e-5
    r = op.residual(dev(lay.faces_to_padded(f, NH)), dev(lay.faces_to_padded(x, NH)), op.face_tensor())
    assert rel_inf(lay.faces_from_padded(r.cpu().numpy(), NH), f - hop.M_rows @ x) <= 1e-12


@pytest.mark.parametrize("reverse", [False, True])
def test_smoother(case, reverse):
    op, vc = case["op"], case["vc"]
    L = vc.levels[0]
    x0, f = rnd(L.op, 4), rnd(L.op, 5)
    xg = dev(lay.faces_to_padded(x0, NH))
    op.smooth(dev(lay.faces_to_padded(f, NH)), xg, sweeps=2, reverse=reverse)
    ref = x0.copy()
    for _ in range(2):
        vc._smooth(L, ref, f, vc.ORDER[::-1] if reverse else vc.ORDER)
    assert rel_inf(lay.faces_from_padded(xg.cpu().numpy(), NH), ref) <= 1e-12


def test_transfers(case):
    op, vc = case["op"], case["vc"]
    nc = tuple(x // 2 for x in NH)
    r = rnd(vc.levels[0].op, 6)
    fc = op.restrict(dev(lay.faces_to_padded(r, NH)), op.face_tensor(level=1))
    assert rel_inf(lay.faces_from_padded(fc.cpu().numpy(), nc), vc.Rt[0] @ r) <= 1e-12
    xc, x0 = rnd(vc.levels[1].op, 7), rnd(vc.levels[0].op, 8)
    xg = dev(lay.faces_to_padded(x0, NH))
    op.prolong_add(dev(lay.faces_to_padded(xc, nc)), xg)
    assert rel_inf(lay.faces_from_padded(xg.cpu().numpy(), NH), x0 + vc.P[0] @ xc) <= 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_vcycle(case, prec):
    op, vc = case["op"], case["vc"]
    dt = torch.float64 if prec == 64 else torch.float32
    f = rnd(vc.levels[0].op, 9)
    x = op.vcycle(dev(lay.faces_to_padded(f, NH), dt), op.face_tensor(dtype=dt))
    tol = 1e-12 if prec == 64 else 5e-5
    assert rel_inf(lay.faces_from_padded(x.double().cpu().numpy(), NH), vc(f)) <= tol


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32"])
def test_eigs(case, mode):
    dm, op, hop = case["dm"], case["op"], case["hop"]
    w_ref, _ = sym.sym_dense_eigs(hop, 4)
    m = dm.SOLVE_FGMRES_MG64 if mode == "fgmres64" else dm.SOLVE_FGMRES_MG32
    P = op.layout(0)["P"]
    vecs = torch.zeros(4 * 3 * P, dtype=torch.float64, device="cuda")
    out = op.eigs(4, tol=1e-10, seed=5, vecs=vecs, solve_mode=m)
    assert out["status"] == 0, out
    assert np.max(abs(out["lam"] - w_ref) / w_ref) <= 1e-10
    # residual of the symmetric pencil recomputed from the downloaded vectors
    K, a = hop.pencil_active()
    V = vecs.cpu().numpy().reshape(4, 3 * P)
    for c in range(4):
        b = lay.faces_from_padded(V[c], NH)[hop.act]
        r = K @ b - out["lam"][c] * a * b
        rho = np.sqrt(np.sum(r * r / a)) / (out["lam"][c] * np.sqrt(np.sum(a * b * b)))
        assert rho <= 2e-10


def test_project_block_matches_single(case):
    """The block projection's CG visits only the cell-vector units holding an
    active cell or a PMC ghost image; with PMC planes it matches the
    single-vector projection, which visits every cell, to rounding."""
    op, hop = case["op"], case["hop"]
    bs = [dev(lay.faces_to_padded(rnd(hop, 30 + q), NH)) for q in range(3)]
    outs = op.project_block(bs, [op.face_tensor() for _ in range(3)], rtol=1e-13)
    for q in range(3):
        one = op.project(bs[q], op.face_tensor(), rtol=1e-13)
        got, ref = outs[q].cpu().numpy(), one.cpu().numpy()
        assert rel_inf(got, ref) <= 1e-12, q
