"""Pins of the learned-correction oracle (network, loss, gradients).

* the FP64 gradient equals central finite differences of the FP64 loss;
* a network whose only nonzero weights sit on one tap is a shifted
  channel mix, written out by hand;
* bfloat16 rounding is round-to-nearest-even on the top 16 bits (values
  from the format's definition), and bf16=False rounds nothing.
"""
import numpy as np
import pytest

from oracle import learned as ln


def rand_case(seed, n=(5, 4, 6)):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    x0 = rng.standard_normal((nz, ny, nx, 10))
    t = rng.standard_normal((nz, ny, nx, 3))
    m = (rng.random((nz, ny, nx, 3)) > 0.2).astype(float)
    w = rng.standard_normal(ln.N_WEIGHTS) * 0.2
    return w, x0, t, m


def test_weight_count():
    assert ln.N_WEIGHTS == 12528


def test_gradient_matches_finite_differences():
    w, x0, t, m = rand_case(0)
    L, g = ln.loss_and_grad(w, x0, t, m)
    rng = np.random.default_rng(1)
    for idx in rng.choice(w.size, 25, replace=False):
        eps = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[idx] += eps
        wm[idx] -= eps
        fd = (ln.loss_and_grad(wp, x0, t, m)[0] - ln.loss_and_grad(wm, x0, t, m)[0]) / (2 * eps)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_one_tap_network_is_a_shifted_mix():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 5, 2))
    W = np.zeros((27, 2, 3))
    t = 1 * 9 + 2 * 3 + 0          # dz = 0, dy = +1, dx = -1
    W[t] = rng.standard_normal((2, 3))
    out = ln.conv(x, W)
    want = np.zeros((3, 4, 5, 3))
    for k in range(3):
        for j in range(4):
            for i in range(5):
                jj, ii = j + 1, i - 1
                if 0 <= jj < 4 and 0 <= ii < 5:
                    want[k, j, i] = x[k, jj, ii] @ W[t]
    assert np.max(abs(out - want)) < 1e-14


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, -2.5, 3.14159265])
    got = ln.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even -> 1 + 2^-6
    assert got.tolist() == [1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 3.140625]
    w, x0, t, m = rand_case(3)
    a = ln.forward(w, x0, bf16_round=False)
    assert np.array_equal(a["x0"], x0)


def test_residual_loss_gradient_matches_finite_differences():
    """Residual loss with a small SPD stand-in for M (a 7-point stencil)."""
    w, x0, t, m = rand_case(4)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(t.shape)

    def M(d):
        out = 7.0 * d
        for ax in range(3):
            out -= np.roll(d, 1, axis=ax) * 0.5 + np.roll(d, -1, axis=ax) * 0.5
        return out

    c = 0.3
    L, g = ln.residual_loss_and_grad(w, x0, r, M, m, c)
    for idx in rng.choice(w.size, 20, replace=False):
        eps = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[idx] += eps
        wm[idx] -= eps
        fd = (ln.residual_loss_and_grad(wp, x0, r, M, m, c)[0]
              - ln.residual_loss_and_grad(wm, x0, r, M, m, c)[0]) / (2 * eps)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_adam_closed_forms():
    """Adam (Kingma & Ba, Algorithm 1) in closed form, not by retyping it:
    * step 1: the bias-corrected moments are g and g^2, so the step is
      lr g / (|g| + eps) -> lr sign(g) as eps -> 0, whatever b1, b2;
    * a constant gradient keeps m_hat = g and v_hat = g^2 at every step
      (bias correction is exact), so every step is the same;
    * gradients g then -g: m_hat_2 = -g (1 - b1) / (1 + b1), v_hat_2 = g^2,
      so the second step is -lr sign(g) (1 - b1) / (1 + b1);
    * with eps = 0 the update is invariant to scaling all gradients by c > 0.
    A missing bias correction, a swapped b1/b2 or a wrong square root fails
    one of these."""
    rng = np.random.default_rng(0)
    g = rng.standard_normal(50) * np.logspace(-3, 3, 50)
    w0 = rng.standard_normal(50)
    z = np.zeros(50)
    lr = 1e-3
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        w1, m1, v1 = ln.adam(w0, g, z, z, 1, lr, b1, b2, eps=0.0)
        assert np.allclose(w0 - w1, lr * np.sign(g), rtol=1e-12, atol=0)
        # constant gradient: the same step every time
        w, m, v = w0, z, z
        for step in range(1, 6):
            w_new, m, v = ln.adam(w, g, m, v, step, lr, b1, b2, eps=0.0)
            assert np.allclose(w - w_new, lr * np.sign(g), rtol=1e-10, atol=0)
            w = w_new
        # g then -g
        w1, m1, v1 = ln.adam(w0, g, z, z, 1, lr, b1, b2, eps=0.0)
        w2, _, _ = ln.adam(w1, -g, m1, v1, 2, lr, b1, b2, eps=0.0)
        assert np.allclose(w2 - w1, lr * np.sign(g) * (1 - b1) / (1 + b1), rtol=1e-10, atol=0)
        # scale invariance
        wa, ma, va = ln.adam(w0, g, z, z, 1, lr, b1, b2, eps=0.0)
        wb, mb, vb = ln.adam(w0, 37.0 * g, z, z, 1, lr, b1, b2, eps=0.0)
        g2 = rng.standard_normal(50)
        wa2, _, _ = ln.adam(wa, g2, ma, va, 2, lr, b1, b2, eps=0.0)
        wb2, _, _ = ln.adam(wb, 37.0 * g2, mb, vb, 2, lr, b1, b2, eps=0.0)
        assert np.allclose(wa2, wb2, rtol=1e-12, atol=1e-15)
    # eps enters only beside sqrt(v_hat): a tiny gradient moves by lr g / eps
    w1, _, _ = ln.adam(w0, 1e-12 * np.ones(50), z, z, 1, lr, eps=1e-8)
    assert np.allclose(w0 - w1, lr * 1e-12 / (1e-12 + 1e-8), rtol=1e-10)
