"""GPU parity of the learned correction against the NumPy oracle.

An ellipsoid on a 20 x 16 x 24 grid (h = 1/20; x rows of 20 cells leave a
ragged 4-cell tail after one 16-cell MFMA segment), fractions from the
oracle.  The library's network (bfloat16 on MFMA, FP32 accumulation) is
compared with ``oracle.learned`` rounding to bfloat16 at the same points:
  * forward correction: max error <= 2e-3 of the largest value;
  * a training pair from the solver satisfies M e = r to 1e-11;
  * error and residual losses to 1e-4, their weight gradients to 2e-3
    (relative 2-norm), the residual loss with the oracle's sparse M, on
    seeded N(0,1) pairs (r, e) on the active faces;
  * two Adam steps (dm_net_train_pairs) against the oracle's Adam step
    (Kingma & Ba) applied to the oracle's own gradients, weight by weight;
  * Adam training lowers the loss; the learned solve mode converges and
    its eigenvalues match the oracle's to 1e-9.
"""
import numpy as np
import pytest

from oracle import eigs as oeigs, geometry as geo, learned as ln, operators as ops
import layout as lay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = (20, 16, 24)
H = 1.0 / 20
SIGMA = 5.0


def cells(vec, n, nch):
    """Padded blocks (nch x P) -> per-cell channels (nz, ny, nx, nch)."""
    a = np.asarray(vec).reshape(nch, n[2] + 2, n[1] + 2, n[0] + 2)[:, 1:-1, 1:-1, 1:-1]
    return np.moveaxis(a, 0, -1)


def static_channels(fr, n):
    nx, ny, nz = n
    ch = [fr["ax"][:, :, :nx], fr["ay"][:, :ny, :], fr["az"][:nz],
          fr["lx"][:nz, :ny, :], fr["ly"][:nz, :, :nx], fr["lz"][:, :ny, :nx], fr["v"]]
    return np.stack(ch, axis=-1)


@pytest.fixture(scope="module")
def case():
    from paper_1301_3794_amd import dm
    g = geo.Ellipsoid((0.5, 0.4, 0.6), (0.42, 0.33, 0.5))
    fr = geo.fractions(g, N, H)
    op = dm.Operator(dm.user_fractions(lay.fractions_to_padded(fr, N)), N, H, SIGMA, levels=3, learned_patience=0)
    net = dm.Net(seed=1)
    w = (np.random.default_rng(11).standard_normal(ln.N_WEIGHTS) * 0.15).astype(np.float32)
    net.set_weights(w)
    net.attach(op)
    stat = static_channels(fr, N)
    mask = (stat[..., :3] > 0).astype(float)
    print("[case] learned ellipsoid", N, flush=True)
    yield dict(dm=dm, op=op, net=net, w=w.astype(np.float64), fr=fr, stat=stat, mask=mask)
    op.close()
    net.close()


def rms(r_cells, mask):
    return float(np.sqrt(np.sum((r_cells * mask) ** 2) / mask.sum()))


def test_forward_matches_oracle(case):
    dm, op = case["dm"], case["op"]
    P = op.layout(0)["P"]
    rng = np.random.default_rng(5)
    r = np.zeros(3 * P)
    act = np.concatenate([case_fr_block(case, c) for c in range(3)]) > 0
    r[act] = rng.standard_normal(act.sum())
    rc = cells(r, N, 3)
    s = rms(rc, case["mask"])
    out = dm.net_apply(op, torch.tensor(r, device="cuda"), op.face_tensor(), scale=s)
    got = cells(out.cpu().numpy(), N, 3)
    x0 = np.concatenate([rc / s, case["stat"]], axis=-1)
    ref = ln.forward(case["w"], x0, bf16_round=True)["y"] * s * H * H * case["mask"]
    err = np.max(abs(got - ref)) / np.max(abs(ref))
    print("forward max rel err", err)
    assert err <= 2e-3


def case_fr_block(case, c):
    """Face fractions of component c as a padded block (library numbering)."""
    name = ("ax", "ay", "az")[c]
    return lay.to_padded(case["fr"][name], N)


@pytest.fixture(scope="module")
def pair(case):
    """A seeded pair (r, e): N(0,1) on the active faces (the losses and
    gradients are defined for any pair)."""
    return seeded_face_vector(case, 7), seeded_face_vector(case, 8)


def seeded_face_vector(case, seed):
    P = case["op"].layout(0)["P"]
    act = np.concatenate([case_fr_block(case, c) for c in range(3)]) > 0
    x = np.zeros(3 * P)
    x[act] = np.random.default_rng(seed).standard_normal(act.sum())
    return torch.tensor(x, device="cuda")


def test_pair_satisfies_M_e_equals_r(case):
    dm, op = case["dm"], case["op"]
    r, e = op.face_tensor(), op.face_tensor()
    dm.net_make_pair(op, 7, r, e)
    me = op.apply(dm.APPLY_M, e, op.face_tensor())
    rel = float((me - r).norm() / r.norm())
    assert rel <= 1e-11 and float(e.norm()) > 0


def test_loss_and_gradient_match_oracle(case, pair):
    dm, op = case["dm"], case["op"]
    r, e = pair
    rc, ec = cells(r.cpu().numpy(), N, 3), cells(e.cpu().numpy(), N, 3)
    s = rms(rc, case["mask"])
    L, g = dm.net_loss_grad(op, r, e, scale=s)
    x0 = np.concatenate([rc / s, case["stat"]], axis=-1)
    t = ec / (s * H * H)
    L_ref, g_ref = ln.loss_and_grad(case["w"], x0, t, case["mask"], bf16_round=True)
    print("loss", L, L_ref, "grad rel", np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    assert L == pytest.approx(L_ref, rel=1e-4)
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) <= 2e-3


def test_residual_loss_and_gradient_match_oracle(case, pair):
    dm, op = case["dm"], case["op"]
    r, _ = pair
    rc = cells(r.cpu().numpy(), N, 3)
    s = rms(rc, case["mask"])
    L, g = dm.net_loss_grad(op, r, None, scale=s, kind=dm.NET_LOSS_RESIDUAL)
    M = cell_operator(case)
    x0 = np.concatenate([rc / s, case["stat"]], axis=-1)
    L_ref, g_ref = ln.residual_loss_and_grad(case["w"], x0, rc, M, case["mask"], s * H * H, bf16_round=True)
    print("residual loss", L, L_ref, "grad rel", np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    assert L == pytest.approx(L_ref, rel=1e-4)
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) <= 2e-3


def cell_operator(case):
    """The oracle's sparse M acting on per-cell channel arrays (nz, ny, nx, 3)."""
    o = ops.build(case["fr"], N, H, SIGMA)
    nx, ny, nz = N

    def M(d):
        fam = {"ax": np.zeros((nz, ny, nx + 1)), "ay": np.zeros((nz, ny + 1, nx)),
               "az": np.zeros((nz + 1, ny, nx))}
        fam["ax"][:, :, :nx] = d[..., 0]
        fam["ay"][:, :ny, :] = d[..., 1]
        fam["az"][:nz] = d[..., 2]
        ax, ay, az = o.grid.split_faces(o.M @ o.grid.face_vector(fam))
        return np.stack([ax[:, :, :nx], ay[:, :ny, :], az[:nz]], axis=-1)
    return M


def test_adam_steps_match_oracle(case):
    """Two Adam steps on two seeded pairs (residual loss) from seeded
    weights: the device's FP32 master weights against the oracle's Adam step
    on the oracle's own gradients.  Step 1 moves each weight by lr sign(g),
    so the bar applies where the gradients are well above the device/oracle
    gradient difference (|g| >= 5e-2 of their RMS in both steps; the
    gradients are heavy-tailed, so that is about two thirds of the
    weights): |w_dev - w_ref| <= 1e-2 lr; every weight stays within 8 lr."""
    dm, op, net = case["dm"], case["op"], case["net"]
    lr = 1e-3
    w0 = (np.random.default_rng(21).standard_normal(ln.N_WEIGHTS) * 0.15).astype(np.float32)
    net.set_weights(w0)                     # also resets the Adam state
    rs = [seeded_face_vector(case, 31), seeded_face_vector(case, 32)]
    try:
        loss = dm.net_train_pairs(op, rs, lr=lr, kind=dm.NET_LOSS_RESIDUAL)
        w_dev = net.weights().astype(np.float64)
    finally:
        net.set_weights(case["w"].astype(np.float32))
    M = cell_operator(case)
    w, m, v = w0.astype(np.float64), np.zeros(ln.N_WEIGHTS), np.zeros(ln.N_WEIGHTS)
    grads = []
    for step, r in enumerate(rs, 1):
        rc = cells(r.cpu().numpy(), N, 3)
        s = rms(rc, case["mask"])
        x0 = np.concatenate([rc / s, case["stat"]], axis=-1)
        L_ref, g = ln.residual_loss_and_grad(w, x0, rc, M, case["mask"], s * H * H, bf16_round=True)
        assert loss[step - 1] == pytest.approx(L_ref, rel=1e-4)
        grads.append(g)
        w, m, v = ln.adam(w, g, m, v, step, lr)
    good = np.ones(ln.N_WEIGHTS, bool)
    for g in grads:
        good &= np.abs(g) >= 5e-2 * np.sqrt(np.mean(g * g))
    d = np.abs(w_dev - w)
    print("adam: well-conditioned fraction", good.mean(), "max dev there / lr", d[good].max() / lr)
    assert good.mean() >= 0.6
    assert d[good].max() <= 1e-2 * lr
    assert d.max() <= 8 * lr


def test_training_lowers_the_loss(case):
    dm, op = case["dm"], case["op"]
    loss = dm.net_train(op, 300, lr=2e-3, seed=100)
    assert np.all(np.isfinite(loss))
    first, last = loss[:30].mean(), loss[-30:].mean()
    print("loss first/last", first, last)
    assert last < 0.8 * first


def test_learned_solve_and_eigenvalues(case):
    dm, op = case["dm"], case["op"]
    f = op.apply(dm.APPLY_A, torch.randn(3 * op.layout(0)["P"], dtype=torch.float64,
                                         generator=torch.Generator().manual_seed(3)).cuda(),
                 op.face_tensor())
    out = op.solve(f, op.face_tensor(), mode=dm.SOLVE_FGMRES_MG32_LEARNED, rtol=1e-10)
    assert out["status"] == 0
    assert out["learned_accepted"] + out["learned_rejected"] == out["iterations"]
    res = op.eigs(4, sigma=SIGMA, tol=1e-10, seed=2, solve_mode=dm.SOLVE_FGMRES_MG32_LEARNED)
    assert res["status"] == 0
    o = ops.build(case["fr"], N, H, SIGMA)
    w_ref = oeigs.lanczos_eigs(o, 4, sigma_o=SIGMA, block=4, tol=1e-11)[0]
    assert np.max(abs(res["lam"] - w_ref) / w_ref) <= 1e-9


def test_learned_patience_stops_rejected_corrections(case):
    """With learned_patience = 1 a solve stops trying the correction after its
    first rejection; an untrained network (its corrections are mostly
    rejected) then leaves the solve to the plain V-cycle.  Same solution as
    the plain FP32-multigrid mode (1e-9)."""
    dm = case["dm"]
    net = dm.Net(seed=5)
    with dm.Operator(dm.user_fractions(lay.fractions_to_padded(case["fr"], N)), N, H, SIGMA, levels=3,
                     learned_patience=1) as op:
        net.attach(op)
        f = op.apply(dm.APPLY_A, seeded_face_vector(case, 41), op.face_tensor())
        x = op.face_tensor()
        out = op.solve(f, x, mode=dm.SOLVE_FGMRES_MG32_LEARNED, rtol=1e-11, maxit=300)
        ref = op.face_tensor()
        op.solve(f, ref, mode=dm.SOLVE_FGMRES_MG32, rtol=1e-11, maxit=300)
        dm.Net.detach(op)
    net.close()
    print("patience 1: accepted", out["learned_accepted"], "rejected", out["learned_rejected"], "its",
          out["iterations"])
    assert out["status"] == 0
    assert out["learned_rejected"] <= 1
    if out["learned_rejected"] == 1:
        assert out["learned_accepted"] + out["learned_rejected"] < out["iterations"] or out["iterations"] <= 1
    assert float((x - ref).abs().max() / ref.abs().max()) <= 1e-9


def test_learned_mode_needs_a_network(case):
    dm, op = case["dm"], case["op"]
    dm.Net.detach(op)
    with pytest.raises(dm.DMError):
        op.solve(op.face_tensor(), op.face_tensor(), mode=dm.SOLVE_FGMRES_MG32_LEARNED)
    with pytest.raises(dm.DMError) as e:
        op.time_kernel(dm.KERNEL_NET, prec=32, level=0, reps=2)
    assert e.value.code == dm.DM_EINVAL
    case["net"].attach(op)
    assert op.time_kernel(dm.KERNEL_NET, prec=32, level=0, reps=2) > 0.0
    with pytest.raises(dm.DMError):
        op.time_kernel(dm.KERNEL_NET, prec=64, level=0, reps=2)
