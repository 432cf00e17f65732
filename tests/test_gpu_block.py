"""GPU parity of the block (multi-right-hand-side) path against the oracle.

The block eigensolver's inversions of one outer step (Sec. 4.3: each
application of T is an inversion of M) share the operator, so the library
solves up to 4 of them in lockstep with block kernels that read each
coefficient once for all vectors.  Checked through the C ABI:
  * dm_vcycle_block, 1..4 vectors, FP64 and FP32, on the 16^3 sphere, the
    ragged 12 x 10 x 14 ellipsoid and the PMC quarter two-cell cavity: every
    vector against the oracle's V-cycle (FP64 1e-12, FP32 5e-5) and against
    the single-vector dm_vcycle (FP64 1e-14, FP32 1e-6);
  * dm_solve_block in the FP64 and FP32 FGMRES modes (the learned mode
    runs through the eigensolver in the learned tests): each system against a sparse
    direct solve of the oracle's M (1e-9), its reported residual <= rtol,
    iteration counts equal to dm_solve's for the same right-hand side, a
    zero right-hand side (converged at once) inside a block;
  * dm_project_block, 1..4 vectors: each against the oracle's projection
    (1e-9) and against dm_project (1e-12), divergence-free to rounding;
  * the eigensolver (which takes the block path for block size 4) still
    matches the oracle's eigenvalues to 1e-10;
  * restarts of FGMRES(4) inside the lockstep, as dm_solve takes them;
  * the FP32 Krylov basis (operator option krylov_basis_f32, FP32 FGMRES
    mode): each system against the sparse direct solve (1e-9) with its true
    residual within the tolerance, under FGMRES(30) and FGMRES(4), and the
    eigensolver's eigenvalues against the oracle (1e-10);
  * both forms of the block smoother's cut-row part (one wavefront per
    vector, and one thread per row looping over the vectors, which the
    full-size grids take) against the oracle's V-cycle, by forcing the loop
    with the operator option cut_wave_split = 0;
  * argument errors: 5 vectors, the PCG mode.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import eigs as oeigs, geometry as geo, multigrid as omg, operators as ops, symmetry as sym
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "sphere16": dict(n=(16, 16, 16), h=1.0 / 16, geom=geo.sphere((0.5, 0.5, 0.5), 0.45), sigma=5.0, levels=3),
    "ragged": dict(n=(12, 10, 14), h=1.0 / 14, geom=geo.Ellipsoid((0.45, 0.36, 0.5), (0.38, 0.31, 0.42)),
                   sigma=3.0, levels=2),
}


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x, dtype=torch.float64):
    return torch.tensor(x, dtype=dtype, device="cuda")


def rnd(act, size, seed):
    x = np.zeros(size)
    x[act] = np.random.default_rng(seed).standard_normal(act.size)
    return x


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_1301_3794_amd import dm
    c = CASES[request.param]
    n, h = c["n"], c["h"]
    fr = geo.fractions(c["geom"], n, h)
    oop = ops.build(fr, n, h, c["sigma"])
    vc = omg.VCycle(fr, n, h, c["sigma"], c["levels"])
    op = dm.Operator(dm.user_fractions(lay.fractions_to_padded(fr, n)), n, h, c["sigma"], levels=c["levels"])
    print(f"[case] block {request.param} n={n}", flush=True)
    yield dict(c, name=request.param, fr=fr, dm=dm, oop=oop, vc=vc, op=op)
    op.close()


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("nr", [1, 2, 3, 4])
def test_vcycle_block(case, prec, nr):
    op, vc, n, oop = case["op"], case["vc"], case["n"], case["oop"]
    dt = torch.float64 if prec == 64 else torch.float32
    fs = [rnd(oop.act, oop.grid.n_faces, 30 + q) for q in range(nr)]
    fd = [dev(lay.faces_to_padded(f, n), dt) for f in fs]
    xs = op.vcycle_block(fd, [op.face_tensor(dtype=dt) for _ in range(nr)])
    for q in range(nr):
        got = lay.faces_from_padded(xs[q].double().cpu().numpy(), n)
        assert rel_inf(got, vc(fs[q])) <= (1e-12 if prec == 64 else 5e-5), q
        one = op.vcycle(fd[q], op.face_tensor(dtype=dt))
        assert rel_inf(got, lay.faces_from_padded(one.double().cpu().numpy(), n)) <= (1e-14 if prec == 64 else 1e-6)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("nr", [2, 3, 4])
def test_vcycle_block_row_loop(case, prec, nr):
    """The block smoother's cut rows by one thread per row looping over the
    vectors (forced: cut_wave_split = 0), the path the 128^3 and 96 x 96 x
    1024 grids take on their finest levels."""
    dm, vc, n, oop = case["dm"], case["vc"], case["n"], case["oop"]
    dt = torch.float64 if prec == 64 else torch.float32
    with dm.Operator(dm.user_fractions(lay.fractions_to_padded(case["fr"], n)), n, case["h"], case["sigma"],
                     levels=case["levels"], cut_wave_split=0) as op:
        fs = [rnd(oop.act, oop.grid.n_faces, 80 + q) for q in range(nr)]
        fd = [dev(lay.faces_to_padded(f, n), dt) for f in fs]
        xs = op.vcycle_block(fd, [op.face_tensor(dtype=dt) for _ in range(nr)])
        for q in range(nr):
            got = lay.faces_from_padded(xs[q].double().cpu().numpy(), n)
            assert rel_inf(got, vc(fs[q])) <= (1e-12 if prec == 64 else 5e-5), q
            one = op.vcycle(fd[q], op.face_tensor(dtype=dt))
            assert rel_inf(got, lay.faces_from_padded(one.double().cpu().numpy(), n)) <= \
                (1e-14 if prec == 64 else 1e-6)


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32"])
def test_solve_block_matches_direct_and_single(case, mode):
    dm, op, oop, n = case["dm"], case["op"], case["oop"], case["n"]
    m = dm.SOLVE_FGMRES_MG64 if mode == "fgmres64" else dm.SOLVE_FGMRES_MG32
    fs = [rnd(oop.act, oop.grid.n_faces, 40 + q) for q in range(4)]
    fs[2] = np.zeros_like(fs[2])                 # converged before the first step
    fd = [dev(lay.faces_to_padded(f, n)) for f in fs]
    xs = [op.face_tensor() for _ in range(4)]
    infos = op.solve_block(fd, xs, mode=m, rtol=1e-11, maxit=300)
    lu = sla.splu(oop.M_a.tocsc())
    for q in range(4):
        assert infos[q]["status"] == 0, infos[q]
        got = lay.faces_from_padded(xs[q].cpu().numpy(), n)
        if q == 2:
            assert infos[q]["iterations"] == 0 and np.all(got == 0)
            continue
        ref = np.zeros_like(fs[q])
        ref[oop.act] = lu.solve(fs[q][oop.act])
        assert rel_inf(got, ref) <= 1e-9, q
        assert infos[q]["rel_residual"] <= 1e-11
        single = op.solve(fd[q], op.face_tensor(), mode=m, rtol=1e-11, maxit=300)
        assert single["iterations"] == infos[q]["iterations"], (q, single, infos[q])


@pytest.mark.parametrize("nr", [1, 3, 4])
def test_project_block(case, nr):
    op, oop, n = case["op"], case["oop"], case["n"]
    bs = [rnd(oop.act, oop.grid.n_faces, 70 + q) for q in range(nr)]
    if nr == 4:
        # an already divergence-free vector beside the others (no CG step)
        bs[3] = np.zeros_like(bs[3])
        bs[3][oop.act] = oeigs.Projector(oop, tol=1e-14)(bs[0][oop.act])
    bd = [dev(lay.faces_to_padded(b, n)) for b in bs]
    outs = op.project_block(bd, [op.face_tensor() for _ in range(nr)], rtol=1e-13)
    for q in range(nr):
        got = lay.faces_from_padded(outs[q].cpu().numpy(), n)
        ref = np.zeros_like(bs[q])
        ref[oop.act] = oeigs.Projector(oop, tol=1e-13)(bs[q][oop.act])
        assert rel_inf(got, ref) <= 1e-9, q
        one = op.project(bd[q], op.face_tensor(), rtol=1e-13)
        assert rel_inf(got, lay.faces_from_padded(one.cpu().numpy(), n)) <= 1e-12, q
        div = oop.D @ (oop.a * got)
        assert np.max(abs(div)) <= 1e-9 * max(np.max(abs(oop.D @ (oop.a * bs[0]))), 1e-300)


def test_solve_block_restarts(case):
    """FGMRES(m) restarts inside the lockstep: with m = 4 a 1e-13 target takes
    several cycles, of different lengths for different systems."""
    dm, oop, n = case["dm"], case["oop"], case["n"]
    op = dm.Operator(dm.user_fractions(lay.fractions_to_padded(case["fr"], n)), n, case["h"], case["sigma"],
                     levels=case["levels"], fgmres_restart=4)
    fs = [rnd(oop.act, oop.grid.n_faces, 50 + q) for q in range(3)]
    fd = [dev(lay.faces_to_padded(f, n)) for f in fs]
    xs = [op.face_tensor() for _ in range(3)]
    infos = op.solve_block(fd, xs, mode=dm.SOLVE_FGMRES_MG32, rtol=1e-13, maxit=400)
    for q in range(3):
        single = op.solve(fd[q], op.face_tensor(), mode=dm.SOLVE_FGMRES_MG32, rtol=1e-13, maxit=400)
        assert infos[q]["restarts"] >= 2
        assert (infos[q]["status"], infos[q]["iterations"], infos[q]["restarts"]) == \
            (single["status"], single["iterations"], single["restarts"])
        r = fs[q][oop.act] - oop.M_a @ lay.faces_from_padded(xs[q].cpu().numpy(), n)[oop.act]
        assert np.linalg.norm(r) <= 2e-13 * np.linalg.norm(fs[q][oop.act])
    op.close()


@pytest.mark.parametrize("restart", [30, 4])
def test_solve_block_fp32_basis(case, restart):
    """The basis stored in FP32: the Arnoldi relation holds to FP32 rounding,
    so the solves restart more, but FGMRES confirms each convergence with the
    FP64 residual: every answer still meets the tolerance."""
    dm, oop, n = case["dm"], case["oop"], case["n"]
    op = dm.Operator(dm.user_fractions(lay.fractions_to_padded(case["fr"], n)), n, case["h"], case["sigma"],
                     levels=case["levels"], fgmres_restart=restart, krylov_basis_f32=1)
    fs = [rnd(oop.act, oop.grid.n_faces, 60 + q) for q in range(4)]
    fs[1] = np.zeros_like(fs[1])
    fd = [dev(lay.faces_to_padded(f, n)) for f in fs]
    xs = [op.face_tensor() for _ in range(4)]
    infos = op.solve_block(fd, xs, mode=dm.SOLVE_FGMRES_MG32, rtol=1e-11, maxit=600)
    lu = sla.splu(oop.M_a.tocsc())
    for q in range(4):
        assert infos[q]["status"] == 0, infos[q]
        got = lay.faces_from_padded(xs[q].cpu().numpy(), n)
        if q == 1:
            assert infos[q]["iterations"] == 0 and np.all(got == 0)
            continue
        ref = np.zeros_like(fs[q])
        ref[oop.act] = lu.solve(fs[q][oop.act])
        assert rel_inf(got, ref) <= 1e-9, q
        r = fs[q][oop.act] - oop.M_a @ got[oop.act]
        assert np.linalg.norm(r) <= 1.5e-11 * np.linalg.norm(fs[q][oop.act]), q
    op.close()


def test_block_eigs_fp32_basis(case):
    dm, oop, n = case["dm"], case["oop"], case["n"]
    op = dm.Operator(dm.user_fractions(lay.fractions_to_padded(case["fr"], n)), n, case["h"], case["sigma"],
                     levels=case["levels"], krylov_basis_f32=1)
    out = op.eigs(4, tol=1e-10, seed=7, block=4, solve_mode=dm.SOLVE_FGMRES_MG32)
    op.close()
    assert out["status"] == 0, out
    lam_ref = oeigs.lanczos_eigs(oop, 4, sigma_o=case["sigma"], block=4, tol=1e-11)[0]
    assert np.max(abs(out["lam"] - lam_ref) / lam_ref) <= 1e-10


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32"])
def test_block_eigs_match_oracle(case, mode):
    dm, op, oop = case["dm"], case["op"], case["oop"]
    m = dm.SOLVE_FGMRES_MG64 if mode == "fgmres64" else dm.SOLVE_FGMRES_MG32
    out = op.eigs(4, tol=1e-10, seed=7, block=4, solve_mode=m)
    assert out["status"] == 0, out
    lam_ref = oeigs.lanczos_eigs(oop, 4, sigma_o=case["sigma"], block=4, tol=1e-11)[0]
    assert np.max(abs(out["lam"] - lam_ref) / lam_ref) <= 1e-10


def test_block_argument_errors(case):
    dm, op = case["dm"], case["op"]
    x = [op.face_tensor() for _ in range(5)]
    with pytest.raises(dm.DMError):
        op.solve_block(x, [op.face_tensor() for _ in range(5)])
    with pytest.raises(dm.DMError):
        op.solve_block(x[:2], [op.face_tensor() for _ in range(2)], mode=dm.SOLVE_PCG64)
    with pytest.raises(dm.DMError):
        op.vcycle_block(x, [op.face_tensor() for _ in range(5)])


def test_block_pmc_vcycle():
    from paper_1301_3794_amd import dm
    H, NH, SIGMA = 1.0 / 16, (8, 8, 24), 2.0
    g = geo.EllipticCells((8 * H, 8 * H), 0.0, 2, 0.4, 0.18, 0.5, 0.25)
    fr_full = geo.fractions(g, (16, 16, 24), H)
    ext = sym.MirrorExtension(NH, H, (0, 1))
    vc = sym.HalfVCycle(fr_full, NH, H, SIGMA, (0, 1), 3)
    fr7 = lay.fractions_to_padded(ext.half_fractions(fr_full), NH)
    for split in (32768, 0):    # cut rows: one wavefront per vector / one thread per row
        with dm.Operator(dm.user_fractions(fr7, bc_lo=(dm.BC_PMC, dm.BC_PMC, dm.BC_PEC)), NH, H, SIGMA,
                         levels=3, cut_wave_split=split) as op:
            hop = vc.levels[0].op
            for prec, dt, tol in ((64, torch.float64, 1e-12), (32, torch.float32, 5e-5)):
                fs = [rnd(hop.act, hop.grid.n_faces, 60 + q) for q in range(3)]
                xs = op.vcycle_block([dev(lay.faces_to_padded(f, NH), dt) for f in fs],
                                     [op.face_tensor(dtype=dt) for _ in range(3)])
                for q in range(3):
                    assert rel_inf(lay.faces_from_padded(xs[q].double().cpu().numpy(), NH), vc(fs[q])) <= tol


def test_time_block_kernel(case):
    dm, op = case["dm"], case["op"]
    for kernel in (dm.KERNEL_APPLY, dm.KERNEL_RESIDUAL, dm.KERNEL_SMOOTH, dm.KERNEL_SWEEP, dm.KERNEL_RESTRICT,
                   dm.KERNEL_PROLONG, dm.KERNEL_VCYCLE):
        for prec in (32, 64):
            assert op.time_block_kernel(kernel, 3, prec=prec, level=0, reps=2) > 0.0
    for bad in (0, 5):
        with pytest.raises(dm.DMError):
            op.time_block_kernel(dm.KERNEL_SWEEP, bad)
