"""Oracle: the geometric V-cycle definition for M (TEST INFRASTRUCTURE ONLY).

The paper preconditions its GMRES inversions of M = C L C^T + A D^T V^-1 D A
- sigma A (eq. discLaplDM) with a multigrid V-cycle, smoothing on every level
on the way down and on the way up (Sec. 6, first paragraph); it used
algebraic multigrid.  This project uses geometric multigrid instead; the
definition below is its reading and is what the GPU V-cycle must reproduce:

* Levels: the cell grid is halved in every direction; the coarse fractions
  are exact sums (means) of the fine ones, i.e. the geometric fractions of
  the coarse grid -- a coarse face is the union of its 4 sub-faces, a coarse
  edge of its 2 sub-edges, a coarse cell of its 8 sub-cells.  The coarse
  operator is M re-discretised with 2h and the same shift.
* Transfers: for the face component normal to axis a, prolongation P is
  piecewise constant across a; along a, a fine face that coincides with a
  coarse face takes its value and a fine face midway between two coarse
  faces takes their mean weighted by the coarse area fractions,
  (a_0 x_0 + a_1 x_1) / (a_0 + a_1) -- the plain mean in vacuum.  The
  weighting keeps a nearly closed coarse face next to a wall normal to it
  from driving the open fine faces beside it (with the plain mean the
  re-discretised coarse correction overshoots such modes by a factor of
  about 45 on a two-cell slice of the elliptic cavity; weighted, about 3).
  Values on inactive faces (a = 0) of either level are dropped.
  Restriction is R = P^T / 8.
* Smoother: Gauss--Seidel in six independent classes, component x colour,
  colour = (i + j + k) mod 2, in the order (x,0) (x,1) (y,0) (y,1) (z,0)
  (z,1) on the way down and the reverse order on the way up, so that the
  V-cycle operator is symmetric.  One class update is
  x_f += (f - M x)_f / M_ff for every face f of the class.
* Coarsest level: exact dense solve on the active faces.

Pinned in tests by: symmetry of the V-cycle operator, exactness with one
level, error contraction, and coarse fractions equal to the fractions
computed directly on the coarse grid.  The numerical values of the V-cycle
themselves have no closed form ("parity unpinned" beyond those properties).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operators as ops


def coarsen_fractions(fr: dict) -> dict:
    """Coarse fractions as means of the fine fractions they contain."""
    ax, ay, az = fr["ax"], fr["ay"], fr["az"]
    lx, ly, lz = fr["lx"], fr["ly"], fr["lz"]
    v = fr["v"]
    out = {}
    # x-face I <- fine x-faces i = 2I, j in {2J,2J+1}, k in {2K,2K+1}
    out["ax"] = 0.25 * (ax[0::2, 0::2, 0::2] + ax[1::2, 0::2, 0::2]
                        + ax[0::2, 1::2, 0::2] + ax[1::2, 1::2, 0::2])
    out["ay"] = 0.25 * (ay[0::2, 0::2, 0::2] + ay[1::2, 0::2, 0::2]
                        + ay[0::2, 0::2, 1::2] + ay[1::2, 0::2, 1::2])
    out["az"] = 0.25 * (az[0::2, 0::2, 0::2] + az[0::2, 1::2, 0::2]
                        + az[0::2, 0::2, 1::2] + az[0::2, 1::2, 1::2])
    out["lx"] = 0.5 * (lx[0::2, 0::2, 0::2] + lx[0::2, 0::2, 1::2])
    out["ly"] = 0.5 * (ly[0::2, 0::2, 0::2] + ly[0::2, 1::2, 0::2])
    out["lz"] = 0.5 * (lz[0::2, 0::2, 0::2] + lz[1::2, 0::2, 0::2])
    out["v"] = 0.125 * sum(v[a::2, b::2, c::2] for a in (0, 1) for b in (0, 1) for c in (0, 1))
    return out


def prolongation(gf: ops.YeeGrid, gc: ops.YeeGrid, mask_f, mask_c, a_c) -> sp.csr_matrix:
    """P (fine faces x coarse faces): area-weighted along the normal, constant
    across it; a_c is the coarse face-fraction vector."""
    R, C, V = [], [], []
    for axis in range(3):
        i, j, k = gf.family(gf.face_shapes[axis])
        fid = gf.face(axis, i, j, k)
        idx = [i, j, k]
        base = [x // 2 for x in idx]
        even = (idx[axis] % 2) == 0
        # even normal index: coincides with a coarse face
        cid = gc.face(axis, *base)
        R.append(fid[even]); C.append(cid[even]); V.append(np.ones(even.sum()))
        # odd normal index: area-weighted mean of the two coarse faces around it
        odd = ~even
        cids, w = [], []
        for shift in (0, 1):
            b2 = list(base)
            b2[axis] = base[axis] + shift
            cid = gc.face(axis, *b2)[odd]
            cids.append(cid)
            w.append(np.where(cid >= 0, a_c[np.maximum(cid, 0)], 0.0))
        tot = w[0] + w[1]
        for cid, wt in zip(cids, w):
            R.append(fid[odd]); C.append(cid)
            V.append(np.where(tot > 0.0, wt / np.where(tot > 0.0, tot, 1.0), 0.0))
    P = ops._coo(R, C, V, (gf.n_faces, gc.n_faces))
    return (sp.diags(mask_f.astype(float)) @ P @ sp.diags(mask_c.astype(float))).tocsr()


class Level:
    def __init__(self, fr, n, h, sigma, grad_div_volume=True):
        self.op = ops.build(fr, n, h, sigma, grad_div_volume)
        self.fr = fr
        self.n = tuple(n)
        self.h = h
        self.M = self.op.M
        d = self.M.diagonal()
        self.active = self.op.a > 0.0
        self.dinv = np.where(self.active, 1.0 / np.where(self.active, d, 1.0), 0.0)
        g = self.op.grid
        # smoothing classes: (component, colour) -> global face ids
        self.classes = {}
        for axis in range(3):
            i, j, k = g.family(g.face_shapes[axis])
            fid = g.face(axis, i, j, k)
            col = (i + j + k) % 2
            for c in (0, 1):
                sel = fid[col == c]
                self.classes[(axis, c)] = sel[self.active[sel]]
        # the rows of M of each class (the same numbers as M[ids], kept once)
        self.class_rows = {key: self.M[ids].tocsr() for key, ids in self.classes.items()}


class VCycle:
    """The V-cycle B ~ M^-1 on the finest level (full face numbering)."""

    ORDER = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]

    def __init__(self, fr, n, h, sigma, levels, nu1=2, nu2=2, grad_div_volume=True, tilde=False):
        """grad_div_volume=False: every level's M without V^-1 (Sec. 6.1
        variant).  tilde=True: the V-cycle built for the symmetric form of
        eq. fullMat2, M~ = A^-1/2 M A^-1/2, written in the variables of M:
        its transfers become P~ = A_f^-1/2 P A_c^1/2 and R~ = P~^T / 8, and
        Gauss--Seidel and the coarsest solve are unchanged by the diagonal
        scaling (Sec. 5.3 variant)."""
        self.nu1, self.nu2 = nu1, nu2
        self.levels = []
        self.P = []
        n = tuple(int(x) for x in n)
        for lev in range(levels):
            if lev:
                if any(x % 2 for x in n):
                    raise ValueError("grid not divisible for coarsening")
                fr = coarsen_fractions(fr)
                n = tuple(x // 2 for x in n)
                h = 2.0 * h
            self.levels.append(Level(fr, n, h, sigma, grad_div_volume))
        for lev in range(levels - 1):
            f, c = self.levels[lev], self.levels[lev + 1]
            P = prolongation(f.op.grid, c.op.grid, f.active, c.active, c.op.a)
            if tilde:
                sf = np.where(f.active, 1.0 / np.sqrt(np.where(f.active, f.op.a, 1.0)), 0.0)
                sc = np.sqrt(np.where(c.active, c.op.a, 0.0))
                P = (sp.diags(sf) @ P @ sp.diags(sc)).tocsr()
            self.P.append(P)
        last = self.levels[-1]
        sel = last.op.act
        self.coarse_sel = sel
        self.coarse_mat = last.M[sel][:, sel].toarray()

    def _smooth(self, L, x, f, order):
        for cls in order:
            ids = L.classes[cls]
            r = f[ids] - L.class_rows[cls] @ x
            x[ids] += r * L.dinv[ids]

    def cycle(self, lev, f):
        L = self.levels[lev]
        if lev == len(self.levels) - 1:
            x = np.zeros_like(f)
            x[self.coarse_sel] = np.linalg.solve(self.coarse_mat, f[self.coarse_sel])
            return x
        x = np.zeros_like(f)
        for _ in range(self.nu1):
            self._smooth(L, x, f, self.ORDER)
        r = f - L.M @ x
        fc = (self.P[lev].T @ r) / 8.0
        x += self.P[lev] @ self.cycle(lev + 1, fc)
        for _ in range(self.nu2):
            self._smooth(L, x, f, self.ORDER[::-1])
        return x

    def __call__(self, f):
        return self.cycle(0, f)

    def apply_active(self, f_act):
        """The V-cycle on an active-face vector of the finest level."""
        L = self.levels[0]
        full = np.zeros(L.op.grid.n_faces)
        full[L.op.act] = f_act
        return self(full)[L.op.act]
