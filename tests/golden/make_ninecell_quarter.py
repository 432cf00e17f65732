"""Writes ninecell_quarter_<nz>_oracle.json: oracle eigenvalues of the 9-cell quarter cavity.

The 9-cell elliptic cavity (tubes 0.1, cells 0.115 long, r_eq 0.103,
r_iris 0.035; length 1.235 along z) on a quarter grid of nxy x nxy x nz
cells with h = 1.235 / nz and nxy = 96 nz / 1024 (the 96 x 96 x 1024
workload's shape at a coarser resolution), perfect-magnetic-conductor planes
x = 0 and y = 0 through the axis (Sec. 6.3), perfect conductors elsewhere.
The 9 smallest nonzero eigenvalues of the symmetric half-cavity pencil by
the oracle's block shift-invert Lanczos on the augmented pencil at the SPD
shift 632, inner CG preconditioned by the oracle's half-cavity V-cycle,
electromagnetic pairs picked by their vanishing divergence.  Calls only
``oracle/``.

Run: python tests/golden/make_ninecell_quarter.py [nz]   (nz = 256: about
half an hour on one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import eigs, geometry as geo, symmetry as sym  # noqa: E402

SIGMA = 632.0
K = 9


def main():
    nz = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    nxy = 96 * nz // 1024
    h = 1.235 / nz
    levels = 4
    t0 = time.time()
    # full mirrored cavity: axis on the middle node line of a 2nxy x 2nxy grid
    g = geo.nine_cell(axis=(nxy * h, nxy * h))
    fr_full = geo.fractions(g, (2 * nxy, 2 * nxy, nz), h)
    print(f"fractions {time.time() - t0:.0f}s", flush=True)
    ext = sym.MirrorExtension((nxy, nxy, nz), h, (0, 1))
    hop = sym.HalfOperators(ext, fr_full, SIGMA)
    pen = sym.SymmetricPencil(hop)
    vc = sym.HalfVCycle(fr_full, (nxy, nxy, nz), h, SIGMA, (0, 1), levels)
    pre = sym.half_vcycle_preconditioner(vc, pen)
    print(f"operators {time.time() - t0:.0f}s, active half faces {pen.a_a.size}", flush=True)
    lam, B, info = eigs.augmented_eigs(pen, K, sigma_o=SIGMA, block=4, tol=1e-11, max_blocks=80,
                                       cg_tol=1e-12, precond=pre,
                                       log=lambda s: print(f"{time.time() - t0:.0f}s {s}", flush=True))
    div = [eigs.div_residual(pen, B[:, c]) for c in range(B.shape[1])]
    out = dict(config=(f"9-cell quarter, {nxy}x{nxy}x{nz} cells, h=1.235/{nz}, PMC x=0 and y=0, "
                       f"shift {SIGMA}"),
               grid=[nxy, nxy, nz], h=h, lam=[float(x) for x in lam],
               residuals=[float(x) for x in info["residuals"]], div_residuals=[float(x) for x in div],
               active_faces=int(pen.a_a.size), n_solves=info["n_solves"], basis=info["dim"],
               seconds=time.time() - t0)
    with open(os.path.join(HERE, f"ninecell_quarter_{nz}_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
