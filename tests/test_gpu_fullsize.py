"""Parity at the full sizes the benchmark runs, on sampled rows.

The library builds the whole operator (128^3 sphere; 96 x 96 x 1024 quarter
9-cell cavity, 6 levels) exactly as ``bench.py`` does and applies M (FP64 and
FP32) and the residual to one seeded random vector.  Sampled 7^3-cell
windows (on the cut surface, where the coefficients are not those of vacuum,
in the interior and at random) are checked in two parts:
  * geometry: the oracle's fractions of the window (a small grid whose cells
    carry the full grid's coordinates) equal the library's full-grid
    fractions there to 1e-12;
  * stencil: the oracle's sparse M, built from the library's fractions of the
    window, times the window's part of the vector, equals the library's
    output on the window's interior faces (whose stencils lie inside the
    window): FP64 1e-12, FP32 2e-5, relative to the largest sampled row.
(Comparing rows built from two independently computed fraction sets mixes
the two: a 1e-13 difference in a small cell's volume is amplified by 1/v.
Shifting the body instead of the cells changes the rounding of the
coordinates, which moves a fraction by ~1e-12 where r'(z) is large.)

Properties at full size: the FP64 V-cycle operator is symmetric,
<u, B v> = <v, B u> to 1e-12; the block V-cycle on the benchmarks' block
sizes (3 vectors on the sphere, 2 on the 9-cell quarter) equals the
single-vector V-cycle on every vector (FP64 1e-14, FP32 1e-6).  At these
sizes the finest level's lists of non-vacuum rows exceed the block
smoother's wave split, so this covers its one-thread-per-row path (the
small grids of the block tests reach it only when it is forced).  And the
9-cell quarter's block FGMRES with its Krylov basis in FP32 meets the
tolerance in the FP64 residual and agrees with the FP64-basis answer; the
128^3 block projection is divergence-free to its tolerance and equals the
single-vector one; the 128^3 transfers satisfy R = P^T / 8 at every level;
and the 128^3 block solves meet their tolerance in the FP64 residual.  At
both sizes the FP32 V-cycle equals the FP64 one to 5e-5.
"""
import numpy as np
import pytest

from oracle import geometry as geo, operators as ops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = 7           # window cells per side
LO, HI = 2, W - 3   # interior cells of a window whose rows are compared


SHAPES = {"ax": (W, W, W + 1), "ay": (W, W + 1, W), "az": (W + 1, W, W),
          "lx": (W + 1, W + 1, W), "ly": (W + 1, W, W + 1), "lz": (W, W + 1, W + 1), "v": (W, W, W)}
NAMES = ("ax", "ay", "az", "lx", "ly", "lz", "v")


def lib_window_fractions(frac7, n_full, origin):
    """The library's fractions (7 padded blocks) on a window, oracle shapes."""
    nx, ny, nz = n_full
    b = np.asarray(frac7).reshape(7, nz + 2, ny + 2, nx + 2)
    i0, j0, k0 = origin
    out = {}
    for q, name in enumerate(NAMES):
        sz, sy, sx = SHAPES[name]
        out[name] = b[q, k0 + 1:k0 + 1 + sz, j0 + 1:j0 + 1 + sy, i0 + 1:i0 + 1 + sx].copy()
    return out


def window_rows(fr, h, sigma, x_full, n_full, origin):
    """Oracle rows M x on the window's interior faces for window fractions fr,
    from the global vector x_full (3 padded blocks of the full grid)."""
    o = ops.build(fr, (W, W, W), h, sigma)
    nx, ny, nz = n_full
    xb = np.asarray(x_full).reshape(3, nz + 2, ny + 2, nx + 2)
    i0, j0, k0 = origin
    fam = {}
    for c, name in enumerate(("ax", "ay", "az")):
        sz, sy, sx = SHAPES[name]
        fam[name] = xb[c, k0 + 1:k0 + 1 + sz, j0 + 1:j0 + 1 + sy, i0 + 1:i0 + 1 + sx].copy()
    y = o.grid.split_faces(o.M @ o.grid.face_vector(fam))
    return [blk[LO:HI + 1, LO:HI + 1, LO:HI + 1] for blk in y]


def lib_rows(y_full, n_full, origin):
    nx, ny, nz = n_full
    yb = np.asarray(y_full).reshape(3, nz + 2, ny + 2, nx + 2)
    i0, j0, k0 = origin
    return [yb[c, k0 + 1 + LO:k0 + 2 + HI, j0 + 1 + LO:j0 + 2 + HI, i0 + 1 + LO:i0 + 2 + HI] for c in range(3)]


def compare(windows, frac7, h, sigma, x, y, n):
    """Relative max difference of the library's rows from the oracle's rows
    (built from the library's window fractions)."""
    worst, scale = 0.0, 0.0
    for o in windows:
        ref = window_rows(lib_window_fractions(frac7, n, o), h, sigma, x, n, o)
        got = lib_rows(y, n, o)
        for a, b in zip(got, ref):
            worst = max(worst, float(np.max(abs(a - b))))
            scale = max(scale, float(np.max(abs(b))))
    assert scale > 0
    return worst / scale


def fraction_gap(windows, geom, frac7, h, n):
    """Max |oracle - library| over the fractions of the windows' interior
    (the window's own wall entities are zero by the oracle's convention)."""
    worst = 0.0
    for o in windows:
        ref = geo.fractions(geom, (W, W, W), h, origin=o)
        got = lib_window_fractions(frac7, n, o)
        for name in NAMES:
            sl = (slice(1, -1),) * 3
            worst = max(worst, float(np.max(abs(ref[name][sl] - got[name][sl]))))
    return worst


def random_vector(P, seed):
    v = np.random.default_rng(seed).standard_normal(3 * P)
    return v


def surface_windows(n, centre, radius, h, count, seed):
    """Window origins whose centre cell is cut by a sphere (or a random cell)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p = np.asarray(centre) + radius * d
        c = np.floor(p / h).astype(int)
        o = tuple(int(v) - W // 2 for v in c)
        if all(0 <= o[a] and o[a] + W <= n[a] for a in range(3)):
            out.append(o)
    return out


@pytest.fixture(scope="module")
def sphere128():
    from paper_1301_3794_amd import dm
    n, h = (128, 128, 128), 1.0 / 128
    op = dm.Operator(dm.sphere((0.5, 0.5, 0.5), 0.45), n, h, 36.0, levels=5)
    P = op.layout(0)["P"]
    x = random_vector(P, 11)
    print("[case] full-size sphere 128^3", flush=True)
    yield dm, op, n, h, x
    op.close()


def test_sphere128_apply_rows(sphere128):
    dm, op, n, h, x = sphere128
    xt = torch.tensor(x, device="cuda")
    y64 = op.apply(dm.APPLY_M, xt, op.face_tensor()).cpu().numpy()
    y32 = op.apply(dm.APPLY_M, xt.float(), op.face_tensor(dtype=torch.float32)).double().cpu().numpy()
    wins = surface_windows(n, (0.5, 0.5, 0.5), 0.45, h, 10, 1) + [(60, 60, 60), (20, 90, 50)]

    fr7 = op.fractions(0)
    assert fraction_gap(wins, geo.sphere((0.5, 0.5, 0.5), 0.45), fr7, h, n) <= 1e-12
    assert compare(wins, fr7, h, 36.0, x, y64, n) <= 1e-12
    x32 = np.asarray(xt.float().double().cpu().numpy())
    assert compare(wins, fr7, h, 36.0, x32, y32, n) <= 2e-5


def test_sphere128_residual_rows(sphere128):
    dm, op, n, h, x = sphere128
    P = op.layout(0)["P"]
    # the residual is that of the active faces: f is zero elsewhere
    fr7 = op.fractions(0)
    f = random_vector(P, 12) * (fr7[:3].reshape(-1) > 0)
    r = op.residual(torch.tensor(f, device="cuda"), torch.tensor(x, device="cuda"), op.face_tensor()).cpu().numpy()
    wins = surface_windows(n, (0.5, 0.5, 0.5), 0.45, h, 6, 2)
    # r = f - M x  <=>  f - r = M x on the sampled rows
    fm = np.asarray(f) - r
    assert compare(wins, fr7, h, 36.0, x, fm, n) <= 1e-12


def test_sphere128_vcycle_symmetric(sphere128):
    dm, op, n, h, _ = sphere128
    P = op.layout(0)["P"]
    a = op.apply(dm.APPLY_A, torch.randn(3 * P, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).cuda(),
                 op.face_tensor())
    b = op.apply(dm.APPLY_A, torch.randn(3 * P, dtype=torch.float64, generator=torch.Generator().manual_seed(4)).cuda(),
                 op.face_tensor())
    Ba = op.vcycle(a, op.face_tensor())
    Bb = op.vcycle(b, op.face_tensor())
    u, v = float(torch.dot(b, Ba)), float(torch.dot(a, Bb))
    assert abs(u - v) <= 1e-12 * max(abs(u), abs(v))


def block_equals_single(op, nr, prec, seed):
    P = op.layout(0)["P"]
    dt = torch.float64 if prec == 64 else torch.float32
    gen = torch.Generator().manual_seed(seed)
    mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
    fs = [(torch.randn(3 * P, dtype=torch.float64, generator=gen) * mask).to(dt).cuda() for _ in range(nr)]
    xs = op.vcycle_block(fs, [op.face_tensor(dtype=dt) for _ in range(nr)])
    worst = 0.0
    for q in range(nr):
        one = op.vcycle(fs[q], op.face_tensor(dtype=dt))
        worst = max(worst, float((xs[q] - one).abs().max() / one.abs().max()))
    return worst


@pytest.mark.parametrize("prec", [64, 32])
def test_sphere128_vcycle_block_equals_single(sphere128, prec):
    dm, op, n, h, _ = sphere128
    assert block_equals_single(op, 3, prec, 5) <= (1e-14 if prec == 64 else 1e-6)


def test_sphere128_project_block(sphere128):
    """The block projection of the benchmark's block size (3 vectors; its
    conjugate gradients over the cell units holding an active cell) at
    128^3: every output divergence-free to the CG's tolerance on the field's
    scale, ||V^-1/2 D A b'|| <= 1e-12 ||b||_A / h, and equal to the
    single-vector projection (which visits every cell) to 1e-12."""
    dm, op, n, h, _ = sphere128
    P = op.layout(0)["P"]
    fr = op.fractions(0)
    a = torch.tensor(fr[:3].reshape(-1), device="cuda")
    v = torch.tensor(fr[6], device="cuda")
    vin = torch.where(v > 0, 1.0 / torch.clamp(v, min=1e-300), torch.zeros_like(v))
    gen = torch.Generator().manual_seed(41)
    mask = torch.tensor(fr[:3].reshape(-1) > 0)
    bs = [(torch.randn(3 * P, dtype=torch.float64, generator=gen) * mask).cuda() for _ in range(3)]
    outs = op.project_block(bs, [op.face_tensor() for _ in range(3)], rtol=1e-13)
    g = op.cell_tensor()
    for q in range(3):
        op.apply(dm.APPLY_DA, outs[q], g)
        div = float(torch.sqrt(torch.sum(g * g * vin)))
        scale = float(torch.sqrt(torch.sum(a * bs[q] * bs[q]))) / h
        assert div <= 1e-12 * scale, (q, div / scale)
        one = op.project(bs[q], op.face_tensor(), rtol=1e-13)
        assert float((outs[q] - one).abs().max() / one.abs().max()) <= 1e-12, q


def fp32_vcycle_gap(op, seed):
    """Largest entry of B32 f - B64 f relative to the largest of B64 f, for a
    seeded random f on the active faces (the FP32 V-cycle of the
    mixed-precision form against the FP64 one)."""
    P = op.layout(0)["P"]
    gen = torch.Generator().manual_seed(seed)
    mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
    f = (torch.randn(3 * P, dtype=torch.float64, generator=gen) * mask).cuda()
    x64 = op.vcycle(f, op.face_tensor())
    x32 = op.vcycle(f.float(), op.face_tensor(dtype=torch.float32))
    return float((x32.double() - x64).abs().max() / x64.abs().max())


def test_sphere128_vcycle_fp32_matches_fp64(sphere128):
    """The FP32 V-cycle of the benchmark equals the FP64 one to FP32
    rounding at 128^3 (5e-5, the small-grid bar against the oracle)."""
    dm, op, n, h, _ = sphere128
    assert fp32_vcycle_gap(op, 53) <= 5e-5


def test_sphere128_transfers_adjoint(sphere128):
    """R = P^T / 8 at every level of the 128^3 hierarchy (FP64):
    <R r, x_c> = <r, P x_c> / 8 for seeded random vectors on the active
    faces, to 1e-12 of the product's scale."""
    dm, op, n, h, _ = sphere128
    gen = torch.Generator().manual_seed(43)
    nlev = op.layout(0)["levels"]
    for lvl in range(nlev - 1):
        mf = torch.tensor(op.fractions(lvl)[:3].reshape(-1) > 0)
        mc = torch.tensor(op.fractions(lvl + 1)[:3].reshape(-1) > 0)
        r = (torch.randn(mf.numel(), dtype=torch.float64, generator=gen) * mf).cuda()
        xc = (torch.randn(mc.numel(), dtype=torch.float64, generator=gen) * mc).cuda()
        rc = op.restrict(r, op.face_tensor(level=lvl + 1), level=lvl)
        px = op.prolong_add(xc, op.face_tensor(level=lvl), level=lvl)
        lhs, rhs = float(torch.dot(rc, xc)), float(torch.dot(r, px)) / 8.0
        scale = float(torch.linalg.norm(rc) * torch.linalg.norm(xc))
        assert abs(lhs - rhs) <= 1e-12 * scale, (lvl, lhs, rhs)


def test_sphere128_block_solve_residual(sphere128):
    """The benchmark's inner solves at 128^3: three systems in lockstep in the
    FP32-multigrid mode to 3e-11 meet the tolerance in the FP64 residual
    recomputed by dm_residual."""
    dm, op, n, h, _ = sphere128
    P = op.layout(0)["P"]
    gen = torch.Generator().manual_seed(47)
    mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
    fs = [(torch.randn(3 * P, dtype=torch.float64, generator=gen) * mask).cuda() for _ in range(3)]
    xs = [op.face_tensor() for _ in range(3)]
    infos = op.solve_block(fs, xs, mode=dm.SOLVE_FGMRES_MG32, rtol=3e-11, maxit=400)
    for q in range(3):
        assert infos[q]["status"] == 0, infos[q]
        r = op.residual(fs[q], xs[q], op.face_tensor())
        assert float(torch.linalg.norm(r) / torch.linalg.norm(fs[q])) <= 4.5e-11, q


@pytest.fixture(scope="module")
def ninecell():
    from paper_1301_3794_amd import dm
    n, h = (96, 96, 1024), 1.235 / 1024
    geom = dm.elliptic_bor((0.0, 0.0), 0.0, 9, 0.103, 0.035, 0.115, 0.1,
                           bc_lo=(dm.BC_PMC, dm.BC_PMC, dm.BC_PEC))
    op = dm.Operator(geom, n, h, 632.0, levels=0)
    P = op.layout(0)["P"]
    x = random_vector(P, 21)
    print("[case] full-size 9-cell quarter 96x96x1024", op.layout(0), flush=True)
    yield dm, op, n, h, x
    op.close()


def test_ninecell_apply_rows(ninecell):
    dm, op, n, h, x = ninecell
    # the stencil reads the PMC ghost layer: give x the mirror images it would hold
    xt = torch.tensor(x, device="cuda")
    y = op.apply(dm.APPLY_M, xt, op.face_tensor()).cpu().numpy()
    g = geo.nine_cell()
    # windows away from the PMC planes (x, y >= 2): an iris, an equator, a tube
    # end plate, a cell wall and the tube; each centred on the cut surface
    zs = [0.1 + 0.115 * 3, 0.1 + 0.115 * 4.5, 0.1, 0.1 + 0.115 * 6.3, 0.05, 1.235 - 0.002]
    wins = []
    for z in zs:
        r = g.radius(z)
        k = int(z / h)
        i = int(r / np.sqrt(2) / h)
        o = (max(2, i - W // 2), max(2, i - W // 2), min(max(0, k - W // 2), n[2] - W))
        wins.append(o)

    fr7 = op.fractions(0)
    assert fraction_gap(wins, g, fr7, h, n) <= 1e-12
    assert compare(wins, fr7, h, 632.0, x, y, n) <= 1e-12


def test_ninecell_vcycle_block_equals_single(ninecell):
    dm, op, n, h, _ = ninecell
    assert block_equals_single(op, 2, 32, 6) <= 1e-6


def test_ninecell_vcycle_fp32_matches_fp64(ninecell):
    dm, op, n, h, _ = ninecell
    assert fp32_vcycle_gap(op, 59) <= 5e-5


def test_empty_geometry_is_rejected():
    """Degenerate input: a cavity smaller than a cell leaves no active face."""
    from paper_1301_3794_amd import dm
    with pytest.raises(dm.DMError) as e:
        dm.Operator(dm.ellipsoid((0.53, 0.51, 0.52), (0.004, 0.004, 0.004)), (16, 16, 16), 1.0 / 16, 5.0)
    assert e.value.code == dm.DM_EINVAL


def test_ninecell_block_solve_fp32_basis():
    """At full size (96 x 96 x 1024, the 9-cell workload's settings: 4 + 4
    sweeps, FGMRES(30), two systems in lockstep) the block FGMRES with its
    Krylov basis stored in FP32 meets the tolerance in the FP64 residual,
    recomputed here by dm_residual, as the FP64-basis solve does; the two
    answers agree to the accuracy the tolerance allows."""
    from paper_1301_3794_amd import dm
    n, h = (96, 96, 1024), 1.235 / 1024
    geom = dm.elliptic_bor((0.0, 0.0), 0.0, 9, 0.103, 0.035, 0.115, 0.1,
                           bc_lo=(dm.BC_PMC, dm.BC_PMC, dm.BC_PEC))
    rtol = 3e-11
    answers = []
    for b32 in (0, 1):
        print(f"[case] full-size 9-cell quarter block solve, FP32 basis {b32}", flush=True)
        with dm.Operator(geom, n, h, 632.0, levels=0, fgmres_restart=30, nu_pre=4, nu_post=4,
                         krylov_basis_f32=b32) as op:
            P = op.layout(0)["P"]
            gen = torch.Generator().manual_seed(31)
            mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
            fs = [(torch.randn(3 * P, dtype=torch.float64, generator=gen) * mask).cuda() for _ in range(2)]
            xs = [op.face_tensor() for _ in range(2)]
            infos = op.solve_block(fs, xs, mode=dm.SOLVE_FGMRES_MG32, rtol=rtol, maxit=800)
            for q in range(2):
                assert infos[q]["status"] == 0, (b32, infos[q])
                r = op.residual(fs[q], xs[q], op.face_tensor())
                rel = float(torch.linalg.norm(r) / torch.linalg.norm(fs[q]))
                assert rel <= 1.5 * rtol, (b32, q, rel)
            answers.append([x.cpu() for x in xs])
    for q in range(2):
        gap = float((answers[0][q] - answers[1][q]).abs().max() / answers[0][q].abs().max())
        assert gap <= 1e-6, (q, gap)
