"""Writes sphere16_oracle.json: oracle eigenvalues of the 16^3 sphere.

Sphere of radius 0.45 centred in the unit cube, 16^3 cells (h = 1/16), the
small workload: the 8 smallest nonzero eigenvalues of the pencil (K, A) on
the active faces by the oracle's dense generalised eigensolve (the plain
definition, no shift, no multigrid), with each pair's eigen-residual and
divergence.  Calls only ``oracle/``.

Run: python tests/golden/make_sphere16.py   (about a minute)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigs, geometry as geo, operators as ops  # noqa: E402


def main():
    n, h, R = (16, 16, 16), 1.0 / 16, 0.45
    t0 = time.time()
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), R), n, h)
    op = ops.build(fr, n, h, 5.0)
    lam, V = eigs.dense_eigs(op, 8)
    out = dict(config="sphere R=0.45 centred in the unit cube, 16^3 cells, h=1/16",
               lam=[float(x) for x in lam],
               residuals=[float(eigs.eig_residual(op, lam[c], V[:, c])) for c in range(len(lam))],
               div_residuals=[float(eigs.div_residual(op, V[:, c])) for c in range(len(lam))],
               active_faces=int(op.act.size), method="dense generalised eigensolve of (K, A)",
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "sphere16_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
