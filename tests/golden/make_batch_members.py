"""Writes batch4_oracle.json: oracle eigenvalues of the 4-ellipsoid test batch.

Four ellipsoids centred in the unit cube (the semi-axes below) on 16^3,
24^3, 32^3 and 40^3 grids (h = 1/N); the 4 smallest nonzero eigenvalues of
each cavity's pencil (K, A) by the oracle's block shift-invert Lanczos at
the SPD shift 5, electromagnetic pairs picked by their vanishing
divergence.  Calls only ``oracle/``.

Run: python tests/golden/make_batch_members.py   (about two minutes)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigs, geometry as geo, operators as ops  # noqa: E402

SEMI = [(0.42, 0.36, 0.31), (0.33, 0.44, 0.38), (0.45, 0.3, 0.4), (0.37, 0.41, 0.46)]
NS = [16, 24, 32, 40]
SIGMA = 5.0


def main():
    members = []
    for s, n in zip(SEMI, NS):
        t0 = time.time()
        fr = geo.fractions(geo.Ellipsoid((0.5, 0.5, 0.5), s), (n, n, n), 1.0 / n)
        op = ops.build(fr, (n, n, n), 1.0 / n, SIGMA)
        lam, B, info = eigs.lanczos_eigs(op, 4, sigma_o=SIGMA, block=4, tol=1e-11)
        members.append(dict(semi_axes=list(s), n=n, lam=[float(x) for x in lam],
                            residuals=[float(eigs.eig_residual(op, lam[c], B[:, c])) for c in range(4)],
                            active_faces=int(op.act.size), seconds=time.time() - t0))
        print(json.dumps(members[-1]), flush=True)
    out = dict(config="4 ellipsoids centred in the unit cube, N^3 cells with h = 1/N, sigma = 5", members=members)
    with open(os.path.join(HERE, "batch4_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
