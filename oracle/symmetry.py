"""Oracle: PMC symmetry planes through the full mirrored cavity (TEST INFRASTRUCTURE ONLY).

Sec. 6.3 runs a quarter of the 9-cell cavity with perfect-magnetic-conductor
planes at x = 0 and y = 0, so that the modes found are those of the whole
cavity that are symmetric under both mirrors.  This module defines that
restriction with nothing but the full-cavity operators of ``operators``:

* the half (or quarter) grid is the upper part of a full grid doubled along
  every PMC axis; the plane is the full grid's middle node plane;
* Q (full faces x half faces) extends a half-cavity field symmetrically: a
  face component normal to the plane is mirrored with sign +1 (B_n even), a
  tangential one with sign -1 (B_t odd, so tangential H vanishes on the
  plane); a face lying in the plane is its own mirror;
* the half-cavity rows of an operator X are R X Q, R selecting each half
  face's own copy; the symmetric pencil is (Q^T K Q, Q^T A Q), whose
  eigenpairs are exactly the full cavity's symmetric ones, and
  Q^T X Q = diag(mult) R X Q with mult the number of copies of each face.

Pinned in tests: the symmetric spectrum is a subset of the full spectrum,
every full eigenvector symmetric under the mirrors is reproduced, and
Q^T M Q = diag(mult) R M Q.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import multigrid as mg
from . import operators as ops


class MirrorExtension:
    """Half grid n_half with low-side PMC planes on `axes` inside the full grid."""

    def __init__(self, n_half, h, axes):
        self.n_half = tuple(int(x) for x in n_half)
        self.axes = tuple(sorted(axes))
        self.n_full = tuple(2 * n if a in self.axes else n for a, n in enumerate(self.n_half))
        self.h = h
        self.gh = ops.YeeGrid(self.n_half, h)
        self.gf = ops.YeeGrid(self.n_full, h)
        shift = [self.n_half[a] if a in self.axes else 0 for a in range(3)]
        self.shift = shift
        rows, cols, vals = [], [], []
        sel_r, sel_c = [], []
        for comp in range(3):
            i, j, k = self.gh.family(self.gh.face_shapes[comp])
            hid = self.gh.face(comp, i, j, k)
            idx = [i, j, k]
            base = [idx[a] + shift[a] for a in range(3)]
            own = self.gf.face(comp, *base)
            sel_r.append(hid)
            sel_c.append(own)
            for flips in itertools.product((False, True), repeat=len(self.axes)):
                fidx = list(base)
                sign = np.ones(hid.size)
                valid = np.ones(hid.size, bool)
                for flip, a in zip(flips, self.axes):
                    if not flip:
                        continue
                    c = self.n_half[a]
                    if comp == a:   # node-centred along a: i -> -i about the plane
                        fidx[a] = 2 * c - fidx[a]
                        valid &= idx[a] > 0          # a face in the plane is its own image
                    else:           # cell-centred along a: i -> -1 - i
                        fidx[a] = 2 * c - 1 - fidx[a]
                        sign = -sign
                fid = self.gf.face(comp, *fidx)
                keep = valid & (fid >= 0)
                rows.append(fid[keep])
                cols.append(hid[keep])
                vals.append(sign[keep])
        self.Q = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(self.gf.n_faces, self.gh.n_faces))
        r = np.concatenate(sel_r)
        c = np.concatenate(sel_c)
        self.R = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(self.gh.n_faces, self.gf.n_faces))
        self.mult = np.asarray((self.Q.T @ self.Q).diagonal())

    def half_fractions(self, fr_full):
        """The half grid's fraction arrays: the full ones on the upper part."""
        sl = [slice(self.shift[a], None) for a in range(3)]
        out = {}
        for name, arr in fr_full.items():
            out[name] = arr[sl[2], sl[1], sl[0]][: arr.shape[0] - self.shift[2],
                                                  : arr.shape[1] - self.shift[1],
                                                  : arr.shape[2] - self.shift[0]].copy()
        return out


class HalfOperators:
    """Half-cavity operators from the full cavity's (one grid level)."""

    def __init__(self, ext: MirrorExtension, fr_full, sigma):
        self.ext = ext
        self.full = ops.build(fr_full, ext.n_full, ext.h, sigma)
        Q, R = ext.Q, ext.R
        self.M_rows = (R @ self.full.M @ Q).tocsr()
        self.K_rows = (R @ self.full.K @ Q).tocsr()
        self.K_sym = (Q.T @ self.full.K @ Q).tocsr()
        self.A_sym = (Q.T @ self.full.A @ Q).tocsr()
        self.a = R @ self.full.a
        self.act = np.flatnonzero(self.a > 0.0)
        self.grid = ext.gh
        self.sigma = sigma

    def pencil_active(self):
        """(K_sym, diag of A_sym) restricted to active half faces."""
        sel = self.act
        return self.K_sym[sel][:, sel].tocsr(), np.asarray(self.A_sym.diagonal())[sel]


def sym_dense_eigs(hop: HalfOperators, k):
    """Smallest nonzero eigenpairs of the symmetric pencil (dense)."""
    import scipy.linalg as sl
    K, a = hop.pencil_active()
    w, V = sl.eigh(K.toarray(), np.diag(a))
    keep = w > 1e-8 * w.max()
    return w[keep][:k], V[:, keep][:, :k]


class _HalfLevel:
    """A V-cycle level whose operator is the half-cavity rows of M."""

    def __init__(self, hop: HalfOperators):
        self.op = hop
        self.M = hop.M_rows
        d = self.M.diagonal()
        self.active = hop.a > 0.0
        self.dinv = np.where(self.active, 1.0 / np.where(self.active, d, 1.0), 0.0)
        g = hop.grid
        self.classes = {}
        for axis in range(3):
            i, j, k = g.family(g.face_shapes[axis])
            fid = g.face(axis, i, j, k)
            col = (i + j + k) % 2
            for c in (0, 1):
                sel = fid[col == c]
                self.classes[(axis, c)] = sel[self.active[sel]]
        self.class_rows = {key: self.M[ids].tocsr() for key, ids in self.classes.items()}


class HalfVCycle(mg.VCycle):
    """The V-cycle definition of ``multigrid`` on the half cavity: Gauss--Seidel
    on the half-cavity rows, transfers P_h = R P Q and R_h = R (P^T / 8) Q
    taken from the full cavity's transfers on symmetric fields."""

    def __init__(self, fr_full, n_half, h, sigma, axes, levels, nu1=2, nu2=2):
        self.nu1, self.nu2 = nu1, nu2
        self.levels, self.P, self.Rt, self.exts = [], [], [], []
        fr, n = fr_full, tuple(n_half)
        for lev in range(levels):
            if lev:
                fr = mg.coarsen_fractions(fr)
                n = tuple(x // 2 for x in n)
                h = 2.0 * h
            ext = MirrorExtension(n, h, axes)
            self.exts.append(ext)
            self.levels.append(_HalfLevel(HalfOperators(ext, fr, sigma)))
        for lev in range(levels - 1):
            ef, ec = self.exts[lev], self.exts[lev + 1]
            Lf, Lc = self.levels[lev], self.levels[lev + 1]
            Pfull = mg.prolongation(ef.gf, ec.gf, Lf.op.full.a > 0, Lc.op.full.a > 0, Lc.op.full.a)
            self.P.append((ef.R @ Pfull @ ec.Q).tocsr())
            self.Rt.append((ec.R @ (Pfull.T / 8.0) @ ef.Q).tocsr())
        last = self.levels[-1]
        sel = last.op.act
        self.coarse_sel = sel
        self.coarse_mat = last.M[sel][:, sel].toarray()

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
        x += self.P[lev] @ self.cycle(lev + 1, self.Rt[lev] @ r)
        for _ in range(self.nu2):
            self._smooth(L, x, f, self.ORDER[::-1])
        return x


class SymmetricPencil:
    """The symmetric half-cavity problem in the form ``eigs.augmented_eigs``
    takes (Sec. 6.3 quarter runs with the grad-div augmented pencil of
    Sec. 5.1): on the active half faces,

        K_a = Q^T K Q,  G_a = Q^T G Q,  A = Q^T A Q = diag(mult * a),
        M_a = K_a + G_a - sigma A,

    and the divergence of a half field b is that of its symmetric extension,
    D A Q b, over the full cavity's active cells (``D_a``, ``v_a``: the
    divergence check ||V^-1/2 D A (Q b)|| / ||b||_A of ``eigs.div_residual``
    with A Q b = Q (a b) written as D_a (a_a b), D_a = D Q diag(1/mult)).
    Its eigenpairs with lambda > 0 are the full cavity's eigenpairs that are
    symmetric under the mirrors (pinned against ``sym_dense_eigs``)."""

    def __init__(self, hop: HalfOperators, sigma=None):
        self.hop = hop
        self.sigma = hop.sigma if sigma is None else sigma
        ext, full = hop.ext, hop.full
        sel = hop.act
        Q = ext.Q[:, sel]
        self.Q_a = Q.tocsr()
        self.mult_a = ext.mult[sel]
        self.K_a = (Q.T @ full.K @ Q).tocsr()
        self.G_a = (Q.T @ full.G @ Q).tocsr()
        self.a_a = self.mult_a * hop.a[sel]
        self.M_a = (self.K_a + self.G_a - self.sigma * sp.diags(self.a_a)).tocsr()
        self.D_a = (full.D[full.cact] @ Q @ sp.diags(1.0 / self.mult_a)).tocsr()
        self.v_a = full.v[full.cact]
        self.act = sel

    def with_shift(self, sigma):
        return SymmetricPencil(self.hop, sigma)


def half_vcycle_preconditioner(vc: HalfVCycle, pencil: SymmetricPencil):
    """M_a^-1 ~ B_h diag(1/mult) on active half faces.  B_h approximates
    (R M Q)^-1 = (diag(1/mult) Q^T M Q)^-1, so B_h diag(1/mult) approximates
    (Q^T M Q)^-1; it is symmetric because diag(mult) B_h is (pinned)."""
    L0 = vc.levels[0]
    n = L0.op.grid.n_faces
    sel = pencil.act
    inv_mult = 1.0 / pencil.mult_a

    def apply(r_act):
        full = np.zeros(n)
        full[sel] = inv_mult * r_act
        return vc(full)[sel]
    return apply
