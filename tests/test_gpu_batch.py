"""Batched cavities: one fused FP32 V-cycle for several operators.

Four ellipsoids in the unit cube on 16^3, 24^3, 32^3 and 40^3 grids
(2, 3, 3 and 4 multigrid levels, so the fused sequence mixes coarsest solves
at different depths), sigma = 5.  Checked:
  * the fused V-cycle gives every member exactly its own V-cycle's values
    (same kernels and arithmetic; compared to 1e-6 of the largest value);
  * dm_batch_eigs (every member's eigensolve on its own thread, every
    preconditioner application fused) gives each member's 4 lowest
    eigenvalues as its own solo eigensolve does (1e-10), and every member's
    as the oracle (1e-10): the 16^3 member's against a live oracle
    eigensolve, all four against the values that
    tests/golden/make_batch_members.py stored from the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import eigs as oeigs, geometry as geo, operators as ops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEMI = [(0.42, 0.36, 0.31), (0.33, 0.44, 0.38), (0.45, 0.3, 0.4), (0.37, 0.41, 0.46)]
NS = [16, 24, 32, 40]
SIGMA = 5.0


@pytest.fixture(scope="module")
def batch():
    from paper_1301_3794_amd import dm
    geoms = [dm.ellipsoid((0.5, 0.5, 0.5), s) for s in SEMI]
    b = dm.Batch(geoms, [(n, n, n) for n in NS], [1.0 / n for n in NS], SIGMA)
    print("[case] batch of", len(NS), "ellipsoids", NS, b.stats(), flush=True)
    yield dm, b
    b.close()


def test_fused_vcycle_equals_member_vcycles(batch):
    dm, b = batch
    fs, refs = [], []
    for q, m in enumerate(b.members):
        P = m.layout(0)["P"]
        v = torch.randn(3 * P, dtype=torch.float64, generator=torch.Generator().manual_seed(q)).cuda()
        f = m.apply(dm.APPLY_A, v, m.face_tensor()).float()
        fs.append(f)
        refs.append(m.vcycle(f.clone(), m.face_tensor(dtype=torch.float32)).clone())
    xs = [torch.zeros_like(f) for f in fs]
    b.vcycle(fs, xs)
    for x, ref in zip(xs, refs):
        scale = float(ref.abs().max())
        assert scale > 0
        assert float((x - ref).abs().max()) <= 1e-6 * scale


def test_batch_eigs_match_solo_and_oracle(batch):
    dm, b = batch
    out = b.eigs(4, sigma=SIGMA, tol=1e-10, seed=5)
    print("batch eigs", out["seconds"], out["inner_iterations"], flush=True)
    assert out["status"] == 0
    assert np.all(out["residuals"] <= 1e-10)
    for q, m in enumerate(b.members):
        solo = m.eigs(4, sigma=SIGMA, tol=1e-10, seed=5, solve_mode=dm.SOLVE_FGMRES_MG32)
        assert solo["status"] == 0
        assert np.max(abs(out["lam"][q] - solo["lam"]) / solo["lam"]) <= 1e-10
    n = NS[0]
    fr = geo.fractions(geo.Ellipsoid((0.5, 0.5, 0.5), SEMI[0]), (n, n, n), 1.0 / n)
    o = ops.build(fr, (n, n, n), 1.0 / n, SIGMA)
    w_ref = oeigs.lanczos_eigs(o, 4, sigma_o=SIGMA, block=4, tol=1e-11)[0]
    assert np.max(abs(out["lam"][0] - w_ref) / w_ref) <= 1e-10
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "batch4_oracle.json")))["members"]
    for q, g in enumerate(gold):
        assert (g["n"], tuple(g["semi_axes"])) == (NS[q], SEMI[q])
        ref = np.array(g["lam"])
        err = float(np.max(abs(out["lam"][q] - ref) / ref))
        print(f"[result] member {q} ({NS[q]}^3) max rel err vs oracle {err:.2e}", flush=True)
        assert err <= 1e-10, (q, err)
