"""Oracle: the electric field of an eigenpair at points (TEST INFRASTRUCTURE ONLY).

Sec. 6.2 compares surface fields with analytic ones by trilinear
interpolation.  In the Yee scheme of Sec. 2 the magnetic eigenvector b on
faces gives the electric field on edges through the Ampere law in the
frequency domain, e = C^T b / k (k^2 = lambda): the Faraday law a b = C L e / k
then closes K b = lambda A b.  Edges outside the cavity (l = 0, e.g. on the
conducting walls) carry e = 0.  Each component is interpolated trilinearly
from its own edge lattice: e_x at ((i + 1/2) h, j h, k h), e_y and e_z
likewise.

Pinned in tests: against the field of a closed-form box mode.
"""
from __future__ import annotations

import math

import numpy as np


def edge_field(op, b_full, lam):
    """e = C^T b / k on every edge (0 where l = 0), split per component into
    arrays [k, j, i] of the edge shapes."""
    e = (op.Ct @ b_full) / math.sqrt(lam)
    e = np.where(op.l > 0.0, e, 0.0)
    g = op.grid
    return [e[g.edge_off[a]:g.edge_off[a + 1]].reshape(g.edge_shapes[a]) for a in range(3)]


def sample_e(op, b_full, lam, points):
    """Trilinear interpolation of each component at the points (n x 3);
    NaN where a stencil leaves the edge lattice."""
    h = op.grid.h
    comps = edge_field(op, b_full, lam)
    out = np.full((len(points), 3), np.nan)
    for q, pt in enumerate(points):
        for c in range(3):
            arr = comps[c]
            shape = (arr.shape[2], arr.shape[1], arr.shape[0])    # (x, y, z) extents
            u = [pt[a] / h - (0.5 if a == c else 0.0) for a in range(3)]
            i0 = [math.floor(x) for x in u]
            if any(i0[a] < 0 or i0[a] + 1 > shape[a] - 1 for a in range(3)):
                continue
            t = [u[a] - i0[a] for a in range(3)]
            v = 0.0
            for dx in (0, 1):
                for dy in (0, 1):
                    for dz in (0, 1):
                        w = ((t[0] if dx else 1 - t[0]) * (t[1] if dy else 1 - t[1])
                             * (t[2] if dz else 1 - t[2]))
                        v += w * arr[i0[2] + dz, i0[1] + dy, i0[0] + dx]
            out[q, c] = v
    return out
