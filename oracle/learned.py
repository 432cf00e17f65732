"""Oracle: the learned correction's network, loss and gradients (TEST INFRASTRUCTURE ONLY).

The paper has no learned component; this is the definition the GPU network
kernels must reproduce.  Plain NumPy, one tap at a time, FP64 arithmetic.

Network (on the cell grid, channels per cell, zero outside the grid):
  X0 (10 ch) -> conv 3^3, 10->16, ReLU -> A1 -> conv 3^3, 16->16, ReLU -> A2
             -> conv 3^3, 16->3 -> Y
  conv:  out[p, o] = sum_{tap, c} in[p + off(tap), c] * W[tap, c, o],
         tap = (dz+1)*9 + (dy+1)*3 + (dx+1), off(tap) = (dx, dy, dz); no bias.
Losses of one pair (mask m on the 3 output channels):
  error loss     L = sum m (Y - T)^2 / sum m T^2 for a target T;
  residual loss  L = |r - M d|^2 / |r|^2 with the correction d = m * Y * c
                 (c the output scale) and M the symmetric operator, given
                 as a callable on per-cell channel arrays; dL/dd =
                 -2 M (r - M d) / |r|^2.

``bf16=True`` rounds, to bfloat16 with round-to-nearest-even, exactly the
quantities the device stores in bfloat16: the input X0, the weights, the
activations A1 and A2, the output gradient dY and the back-propagated
activation gradients dA2 and dA1.  Sums are taken in FP64 here (FP32 on the
device).

Pinned in tests: the FP64 gradients equal central finite differences of the
FP64 loss; a one-tap network equals a shifted channel mix; with bf16=False
nothing is rounded.
"""
from __future__ import annotations

import numpy as np

SHAPES = ((10, 16), (16, 16), (16, 3))          # (in, out) channels per layer
N_WEIGHTS = sum(27 * a * b for a, b in SHAPES)   # 12528


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def taps():
    return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def unpack(w):
    """Flat weight vector -> [W1 (27,10,16), W2 (27,16,16), W3 (27,16,3)]."""
    out, o = [], 0
    for a, b in SHAPES:
        out.append(np.asarray(w[o:o + 27 * a * b], dtype=np.float64).reshape(27, a, b))
        o += 27 * a * b
    return out


def _shift(x, dx, dy, dz):
    """y[k, j, i] = x[k + dz, j + dy, i + dx], zero outside.  x is (nz, ny, nx, C)."""
    nz, ny, nx = x.shape[:3]
    y = np.zeros_like(x)
    ks, js, is_ = [slice(max(0, -d), n - max(0, d)) for d, n in ((dz, nz), (dy, ny), (dx, nx))]
    kt, jt, it = [slice(max(0, d), n - max(0, -d)) for d, n in ((dz, nz), (dy, ny), (dx, nx))]
    y[ks, js, is_] = x[kt, jt, it]
    return y


def conv(x, W):
    """out[p, o] = sum_tap sum_c x[p + off, c] W[tap, c, o]."""
    out = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, (dx, dy, dz) in enumerate(taps()):
        out += np.einsum("kjic,co->kjio", _shift(x, dx, dy, dz), W[t])
    return out


def conv_data_grad(d, W):
    """Gradient of sum(conv(x, W) * g) w.r.t. x for output gradient d."""
    out = np.zeros(d.shape[:3] + (W.shape[1],))
    for t, (dx, dy, dz) in enumerate(taps()):
        out += np.einsum("kjio,co->kjic", _shift(d, -dx, -dy, -dz), W[t])
    return out


def conv_weight_grad(x, d):
    """Gradient of sum(conv(x, W) * d) w.r.t. W."""
    g = np.zeros((27, x.shape[3], d.shape[3]))
    for t, (dx, dy, dz) in enumerate(taps()):
        g[t] = np.einsum("kjic,kjio->co", _shift(x, dx, dy, dz), d)
    return g


def forward(w, x0, bf16_round=False):
    R = bf16 if bf16_round else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3 = [R(m) for m in unpack(w)]
    x0 = R(x0)
    a1 = R(np.maximum(conv(x0, W1), 0.0))
    a2 = R(np.maximum(conv(a1, W2), 0.0))
    y = conv(a2, W3)
    return dict(x0=x0, a1=a1, a2=a2, y=y, W=(W1, W2, W3))


def loss(y, t, m):
    return float(np.sum(m * (y - t) ** 2) / np.sum(m * t * t))


def loss_and_grad(w, x0, t, m, bf16_round=False):
    """Error loss of one pair and its gradient w.r.t. the flat weight vector."""
    R = bf16 if bf16_round else (lambda v: np.asarray(v, dtype=np.float64))
    f = forward(w, x0, bf16_round)
    L = loss(f["y"], t, m)
    dy = R(2.0 * m * (f["y"] - t) / np.sum(m * t * t))
    return L, _backward(f, dy, R)


def _backward(f, dy, R):
    W1, W2, W3 = f["W"]
    g3 = conv_weight_grad(f["a2"], dy)
    d2 = R(conv_data_grad(dy, W3) * (f["a2"] > 0))
    g2 = conv_weight_grad(f["a1"], d2)
    d1 = R(conv_data_grad(d2, W2) * (f["a1"] > 0))
    g1 = conv_weight_grad(f["x0"], d1)
    return np.concatenate([g1.ravel(), g2.ravel(), g3.ravel()])


def residual_loss_and_grad(w, x0, r, M, m, c, bf16_round=False):
    """Residual loss of one pair and its gradient w.r.t. the weights; r and
    M(.) live on per-cell channel arrays (nz, ny, nx, 3)."""
    R = bf16 if bf16_round else (lambda v: np.asarray(v, dtype=np.float64))
    f = forward(w, x0, bf16_round)
    d = m * f["y"] * c
    r3 = r - M(d)
    rr = float(np.sum(r * r))
    L = float(np.sum(r3 * r3)) / rr
    dd = -2.0 * M(r3) / rr
    dy = R(dd * m * c)
    return L, _backward(f, dy, R)


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) of FP32 master weights."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
