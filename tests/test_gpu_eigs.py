"""GPU eigensolve parity on the small configuration and the PEC box.

Small configuration: sphere R = 0.45 centred in the unit cube, 16^3 cells,
sigma = 5, 3-level V-cycle with 2 + 2 red-black sweeps, the 4 lowest
nonzero eigenpairs to rho <= 1e-10.  The library computes its own
fractions; the oracle computes its own.  Bars: eigenvalues within 1e-10
relative of the oracle (FP64 and FP32-multigrid forms), rho recomputed by
the oracle from the downloaded vectors, the exact TM11 triplet degeneracy,
and the closed-form box spectrum.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import eigs as oeigs, geometry as geo, operators as ops
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 16
H = 1.0 / N


@pytest.fixture(scope="module")
def oracle_small():
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), (N, N, N), H)
    oop = ops.build(fr, (N, N, N), H, 5.0)
    lam, _, _ = oeigs.lanczos_eigs(oop, 4, sigma_o=5.0, block=4, tol=1e-12)
    return oop, lam


@pytest.mark.parametrize("mode", ["fgmres64", "fgmres32", "pcg64"])
def test_small_config_eigs(oracle_small, mode):
    from paper_1301_3794_amd import dm
    oop, lam_ref = oracle_small
    m = {"fgmres64": dm.SOLVE_FGMRES_MG64, "fgmres32": dm.SOLVE_FGMRES_MG32, "pcg64": dm.SOLVE_PCG64}[mode]
    print(f"[eigs] sphere16 mode={mode}", flush=True)
    with dm.Operator(dm.sphere((0.5, 0.5, 0.5), 0.45), (N, N, N), H, 5.0, levels=3) as op:
        P = op.layout(0)["P"]
        vecs = torch.zeros(4 * 3 * P, dtype=torch.float64, device="cuda")
        out = op.eigs(4, tol=1e-10, seed=1301, vecs=vecs, solve_mode=m)
    assert out["status"] == 0, out
    lam = out["lam"]
    assert np.max(abs(lam - lam_ref) / lam_ref) <= 1e-10
    assert np.max(out["residuals"]) <= 1e-10
    # TM11: exact triplet on the node-centred grid
    assert (lam[2] - lam[0]) / lam[0] <= 1e-12
    V = vecs.cpu().numpy().reshape(4, 3 * P)
    B = np.stack([lay.faces_from_padded(V[c], (N, N, N))[oop.act] for c in range(4)], axis=1)
    for c in range(4):
        assert oeigs.eig_residual(oop, lam[c], B[:, c]) <= 2e-10
        assert oeigs.div_residual(oop, B[:, c]) <= 1e-9
    G = B.T @ (oop.a_a[:, None] * B)
    assert np.max(abs(G - np.eye(4))) <= 1e-10


def test_box_closed_form_gpu():
    from paper_1301_3794_amd import dm
    n = 16
    h = 1.0 / n
    # closed form; multiplicity 2 when all three indices are nonzero
    vals = []
    for m in itertools.product(range(4), repeat=3):
        if sum(x > 0 for x in m) < 2:
            continue
        lam = sum((2 * math.sin(math.pi * x / (2 * n)) / h) ** 2 for x in m)
        vals += [lam] * (2 if all(x > 0 for x in m) else 1)
    vals = np.sort(vals)[:5]
    with dm.Operator(dm.box(), (n, n, n), h, 5.0, levels=3) as op:
        out = op.eigs(5, tol=1e-10, seed=7)
    assert out["status"] == 0, out
    assert np.max(abs(out["lam"] - vals) / vals) <= 1e-10
