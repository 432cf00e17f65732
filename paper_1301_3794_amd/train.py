"""Training driver of the learned correction: solver-generated pairs on
random ellipsoidal cavities (argument marshalling and the loop only; pairs,
forward, backward and Adam run in the library's kernels).

Recipe: ``count`` ellipsoids centred in the unit cube with semi-axes drawn
uniformly from [0.3, 0.48] (NumPy generator seeded by ``seed``), ``n``^3
cells, shift ``sigma``; each round visits every cavity for ``steps`` Adam
steps on fresh pairs; the learning rate halves at a third and at two thirds
of the rounds.
"""
from __future__ import annotations

import time

import numpy as np

from . import dm


def random_ellipsoids(count, seed=0):
    rng = np.random.default_rng(seed)
    return [tuple(float(a) for a in rng.uniform(0.3, 0.48, 3)) for _ in range(count)]


def train_on_ellipsoids(net: dm.Net, n=64, count=6, steps=200, rounds=5, lr=1e-3, sigma=5.0,
                        seed=0, kind=dm.NET_LOSS_RESIDUAL, verbose=False):
    t0 = time.time()
    ops = [dm.Operator(dm.ellipsoid((0.5, 0.5, 0.5), semi), (n, n, n), 1.0 / n, sigma)
           for semi in random_ellipsoids(count, seed)]
    t_setup = time.time() - t0
    history = []
    try:
        for rd in range(rounds):
            rate = lr * 0.5 ** (rd * 3 // rounds)
            losses = []
            for q, op in enumerate(ops):
                net.attach(op)
                losses.append(dm.net_train(op, steps, lr=rate, seed=10000 + 1000 * rd + 100000 * q,
                                           kind=kind))
            ls = np.concatenate(losses)
            history.append(float(ls.mean()))
            if verbose:
                print(f"  round {rd}: lr {rate:.2e} mean loss {ls.mean():.4f}", flush=True)
    finally:
        for op in ops:
            op.close()
    return dict(loss_per_round=history, pairs=count * steps * rounds, setup_s=t_setup,
                train_s=time.time() - t0 - t_setup)
