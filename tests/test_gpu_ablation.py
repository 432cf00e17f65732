"""Solver-sensitivity variants (Sec. 6.1 and Sec. 5.3) against the oracle, and
the study of their inner-iteration counts.

Parity on the 16^3 sphere (R = 0.45, sigma = 5, 3 levels):
  * V^-1 left out of the grad-div term on every level (grad_div_volume = 0):
    M x and the FP64 V-cycle against the oracle's operator and V-cycle built
    without V^-1 (1e-12);
  * the tilde form's V-cycle (tilde_transfers = 1, eq. fullMat2): FP64 and
    FP32 against the oracle's tilde V-cycle (1e-12, 5e-5), which is pinned on
    the CPU as the plain V-cycle of A^-1/2 M A^-1/2;
  * volume errors of eq. volPert1 on the cut cells (eps = 1): M x against
    the oracle's M from the same perturbed fractions (1e-12), and the
    eigenvalues equal the unperturbed oracle eigenvalues (1e-10): the volumes
    do not enter the electromagnetic modes (Sec. 5.1);
  * the entry points that do not support the tilde form refuse it.
The study (sphere R = 0.49 at 32^3 as in Sec. 6.1, FGMRES(40) to 1e-6,
FP64 V-cycle): average inner iterations of the method and each variant are
printed; the volume errors raise them monotonically in eps.
"""
import numpy as np
import pytest

from oracle import eigs as oeigs, geometry as geo, multigrid as omg, operators as ops
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = (16, 16, 16)
H = 1.0 / 16
SIGMA = 5.0


@pytest.fixture(scope="module")
def base():
    from paper_1301_3794_amd import dm
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), N, H)
    print("[case] ablation variants, sphere 16^3", flush=True)
    return dm, fr


def rnd(oop, seed):
    x = np.zeros(oop.grid.n_faces)
    x[oop.act] = np.random.default_rng(seed).standard_normal(oop.act.size)
    return x


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def dev(x, dt=torch.float64):
    return torch.tensor(lay.faces_to_padded(x, N), dtype=dt, device="cuda")


def test_without_volumes_matches_oracle(base):
    dm, fr = base
    oop = ops.build(fr, N, H, SIGMA, grad_div_volume=False)
    vc = omg.VCycle(fr, N, H, SIGMA, 3, grad_div_volume=False)
    with dm.Operator(dm.user_fractions(lay.fractions_to_padded(fr, N)), N, H, SIGMA, levels=3,
                     grad_div_volume=0) as op:
        x = rnd(oop, 1)
        y = op.apply(dm.APPLY_M, dev(x), op.face_tensor())
        assert rel_inf(lay.faces_from_padded(y.cpu().numpy(), N), oop.M @ x) <= 1e-12
        f = rnd(oop, 2)
        z = op.vcycle(dev(f), op.face_tensor())
        assert rel_inf(lay.faces_from_padded(z.cpu().numpy(), N), vc(f)) <= 1e-12


@pytest.mark.parametrize("prec", [64, 32])
def test_tilde_vcycle_matches_oracle(base, prec):
    dm, fr = base
    vc = omg.VCycle(fr, N, H, SIGMA, 3, tilde=True)
    dt = torch.float64 if prec == 64 else torch.float32
    with dm.Operator(dm.user_fractions(lay.fractions_to_padded(fr, N)), N, H, SIGMA, levels=3,
                     tilde_transfers=1) as op:
        f = rnd(vc.levels[0].op, 3)
        z = op.vcycle(dev(f, dt), op.face_tensor(dtype=dt))
        assert rel_inf(lay.faces_from_padded(z.double().cpu().numpy(), N), vc(f)) <= (1e-12 if prec == 64 else 5e-5)


def test_tilde_form_refused_where_unsupported(base):
    dm, fr = base
    with dm.Operator(dm.sphere((0.5, 0.5, 0.5), 0.45), N, H, SIGMA, levels=3, tilde_transfers=1) as op:
        x = [op.face_tensor() for _ in range(2)]
        for call in (lambda: op.eigs(2), lambda: op.vcycle_block(x, [op.face_tensor() for _ in range(2)]),
                     lambda: op.solve_block(x, [op.face_tensor() for _ in range(2)])):
            with pytest.raises(dm.DMError) as e:
                call()
            assert e.value.code == dm.DM_EINVAL


def test_volume_errors_keep_the_eigenvalues(base):
    from paper_1301_3794_amd import studies
    dm, fr = base
    fr7 = studies.perturb_volumes(lay.fractions_to_padded(fr, N), "log", 1.0, 7)
    frp = lay.fractions_from_padded(fr7, N)
    assert np.max(abs(frp["v"] - fr["v"])) > 0.1
    oop = ops.build(frp, N, H, SIGMA)
    lam_ref = oeigs.lanczos_eigs(ops.build(fr, N, H, SIGMA), 4, sigma_o=SIGMA, block=4, tol=1e-12)[0]
    with dm.Operator(dm.user_fractions(fr7), N, H, SIGMA, levels=3) as op:
        x = rnd(oop, 4)
        y = op.apply(dm.APPLY_M, dev(x), op.face_tensor())
        assert rel_inf(lay.faces_from_padded(y.cpu().numpy(), N), oop.M @ x) <= 1e-12
        out = op.eigs(4, tol=1e-10, seed=5, solve_mode=dm.SOLVE_FGMRES_MG64, max_restarts=40)
    assert out["status"] == 0
    assert np.max(abs(out["lam"] - lam_ref) / lam_ref) <= 1e-10


def test_solver_sensitivity_study():
    from paper_1301_3794_amd import studies
    st = studies.solver_sensitivity(n=32)
    for r in st["rows"]:
        print(f"  {r['variant']:40s} {str(r['value']):8s} avg its {r['avg_iterations']:8.1f} "
              f"converged {r['converged']}", flush=True)
    rows = st["rows"]
    assert rows[0]["variant"] == "method" and rows[0]["converged"]
    eps = [r for r in rows if "volPert1" in r["variant"]]
    assert [r["value"] for r in eps] == [0.1, 0.3, 0.5, 1.0, 2.0, 3.0]
    assert eps[-1]["avg_iterations"] > eps[0]["avg_iterations"]
    assert eps[0]["avg_iterations"] >= rows[0]["avg_iterations"] - 1
