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
