"""Writes sphere128_oracle.json: oracle eigenvalues of the 128^3 sphere.

Sphere of radius 0.45 centred in the unit cube, 128^3 cells (h = 1/128);
the 8 smallest nonzero eigenvalues of (K, A) (TM11 x3 and TM21 x5) by the
oracle's block shift-invert Lanczos on the augmented pencil (K + G, A) at
the SPD shift 5, inner CG preconditioned by the oracle V-cycle (5 levels),
electromagnetic pairs picked by their vanishing divergence.  Calls only
``oracle/``.

Run: python tests/golden/make_sphere128.py   (about an hour on 8 cores)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import eigs, geometry as geo, multigrid as mg  # noqa: E402


def main():
    n, h, R, sig = (128, 128, 128), 1.0 / 128, 0.45, 5.0
    t0 = time.time()
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), R), n, h)
    print(f"fractions {time.time() - t0:.0f}s", flush=True)
    vc = mg.VCycle(fr, n, h, sig, 5)
    op = vc.levels[0].op
    print(f"operators {time.time() - t0:.0f}s, active faces {op.act.size}", flush=True)
    lam, B, info = eigs.augmented_eigs(op, 8, sigma_o=sig, block=4, tol=1e-11, max_blocks=60,
                                       cg_tol=1e-12, precond=vc.apply_active,
                                       log=lambda s: print(f"{time.time() - t0:.0f}s {s}", flush=True))
    div = [eigs.div_residual(op, B[:, c]) for c in range(B.shape[1])]
    out = dict(config="sphere R=0.45 centred in the unit cube, 128^3 cells, h=1/128",
               lam=[float(x) for x in lam], residuals=[float(x) for x in info["residuals"]],
               div_residuals=[float(x) for x in div], active_faces=int(op.act.size),
               n_solves=info["n_solves"], basis=info["dim"], seconds=time.time() - t0)
    with open(os.path.join(HERE, "sphere128_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
