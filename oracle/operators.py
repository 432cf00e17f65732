"""Oracle: staggered Yee operators of the Dey--Mittra method (TEST INFRASTRUCTURE ONLY).

Every matrix is assembled entry by entry from the paper's stencils:

* ``curl_t`` is C^T, faces -> edges: the circulation of b around each edge,
  divided by h.  Its transpose C maps edge values back to faces exactly as
  in eq. farInt: (C w)_x[i,j,k] = (w_y[i,j,k] - w_y[i,j,k+1]
  + w_z[i,j+1,k] - w_z[i,j,k]) / h  (Sec. 2).
* ``div`` is D, faces -> cells: eq. divB (Sec. 4.2); the Dey--Mittra
  divergence is V^-1 D A (eqs. divBInt, divBDM, Sec. 5.1).  The gradient
  is -D^T (eq. gradPhi).
* K = C L C^T (eq. discWaveBDM multiplied by A), G = A D^T V^-1 D A,
  M = K + G - sigma A (eq. discLaplDM), S = D A D^T (eq. proj).

Unknown numbering (internal to the oracle): x-faces, then y-faces, then
z-faces, each block in C order of its [k, j, i] array (x fastest); edges
likewise; cells [k, j, i].  Shapes are those of ``oracle.geometry``.

Pinned in tests: D C = 0 exactly (Sec. 4.2 text after eq. divB), symmetry
and semi-definiteness, the closed-form spectrum of the PEC box, the
decoupling of K + G into three scalar Laplacians in vacuum, the spectrum
partition spec(K+G, A) = spec+(K, A) U spec+(S, V) (Sec. 5.1 text after
eq. discLaplBDM) and face/edge duality of the nonzero spectrum.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .geometry import EDGE_SHAPES, FACE_SHAPES


@dataclass
class YeeGrid:
    n: tuple
    h: float

    def __post_init__(self):
        nx, ny, nz = self.n = tuple(int(x) for x in self.n)
        self.face_shapes = [FACE_SHAPES[s](self.n) for s in ("ax", "ay", "az")]
        self.edge_shapes = [EDGE_SHAPES[s](self.n) for s in ("lx", "ly", "lz")]
        self.cell_shape = (nz, ny, nx)
        self.face_off = np.cumsum([0] + [int(np.prod(s)) for s in self.face_shapes])
        self.edge_off = np.cumsum([0] + [int(np.prod(s)) for s in self.edge_shapes])
        self.n_faces = int(self.face_off[-1])
        self.n_edges = int(self.edge_off[-1])
        self.n_cells = int(np.prod(self.cell_shape))

    # global ids; arguments are integer arrays (i, j, k); out-of-range -> -1
    def _id(self, shape, off, i, j, k):
        ok = (i >= 0) & (j >= 0) & (k >= 0) & (i < shape[2]) & (j < shape[1]) & (k < shape[0])
        gid = off + i + shape[2] * (j + shape[1] * k)
        return np.where(ok, gid, -1)

    def face(self, axis, i, j, k):
        return self._id(self.face_shapes[axis], self.face_off[axis], i, j, k)

    def edge(self, axis, i, j, k):
        return self._id(self.edge_shapes[axis], self.edge_off[axis], i, j, k)

    def cell(self, i, j, k):
        return self._id(self.cell_shape, 0, i, j, k)

    def family(self, shape):
        k, j, i = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]),
                              np.arange(shape[2]), indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    # flatten / unflatten fraction dictionaries into global vectors
    def face_vector(self, fr):
        return np.concatenate([fr[s].ravel() for s in ("ax", "ay", "az")])

    def edge_vector(self, fr):
        return np.concatenate([fr[s].ravel() for s in ("lx", "ly", "lz")])

    def split_faces(self, vec):
        return [vec[self.face_off[a]:self.face_off[a + 1]].reshape(self.face_shapes[a])
                for a in range(3)]


def _coo(rows, cols, vals, shape):
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    keep = (rows >= 0) & (cols >= 0)
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=shape)


def curl_t(g: YeeGrid) -> sp.csr_matrix:
    """C^T: edge circulations of the face field, divided by h."""
    R, C, V = [], [], []
    inv_h = 1.0 / g.h

    def put(e, f, s):
        R.append(e)
        C.append(f)
        V.append(np.full(e.shape, s * inv_h))

    # e_x[i,j,k]: + b_z[i,j,k] - b_z[i,j-1,k] - b_y[i,j,k] + b_y[i,j,k-1]
    i, j, k = g.family(g.edge_shapes[0])
    e = g.edge(0, i, j, k)
    put(e, g.face(2, i, j, k), +1)
    put(e, g.face(2, i, j - 1, k), -1)
    put(e, g.face(1, i, j, k), -1)
    put(e, g.face(1, i, j, k - 1), +1)
    # e_y[i,j,k]: + b_x[i,j,k] - b_x[i,j,k-1] - b_z[i,j,k] + b_z[i-1,j,k]
    i, j, k = g.family(g.edge_shapes[1])
    e = g.edge(1, i, j, k)
    put(e, g.face(0, i, j, k), +1)
    put(e, g.face(0, i, j, k - 1), -1)
    put(e, g.face(2, i, j, k), -1)
    put(e, g.face(2, i - 1, j, k), +1)
    # e_z[i,j,k]: + b_y[i,j,k] - b_y[i-1,j,k] - b_x[i,j,k] + b_x[i,j-1,k]
    i, j, k = g.family(g.edge_shapes[2])
    e = g.edge(2, i, j, k)
    put(e, g.face(1, i, j, k), +1)
    put(e, g.face(1, i - 1, j, k), -1)
    put(e, g.face(0, i, j, k), -1)
    put(e, g.face(0, i, j - 1, k), +1)
    return _coo(R, C, V, (g.n_edges, g.n_faces))


def div(g: YeeGrid) -> sp.csr_matrix:
    """D: net outward face sum per cell divided by h (eq. divB)."""
    i, j, k = g.family(g.cell_shape)
    c = g.cell(i, j, k)
    R, C, V = [], [], []
    for axis, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        R += [c, c]
        C += [g.face(axis, i + di, j + dj, k + dk), g.face(axis, i, j, k)]
        V += [np.full(c.shape, 1.0 / g.h), np.full(c.shape, -1.0 / g.h)]
    return _coo(R, C, V, (g.n_cells, g.n_faces))


@dataclass
class DMOperators:
    """All oracle matrices for one grid, fraction set and shift.

    ``act`` is the index array of active faces (a > 0), ``cact`` of active
    cells (v > 0).  Matrices with suffix ``_a`` are restricted to active
    faces (rows and columns), ``S_a`` to active cells.
    """

    grid: YeeGrid
    fr: dict
    sigma: float
    # False: the grad-div term without V^-1, A D^T D A (the solver-sensitivity
    # variant of Sec. 6.1 that leaves the inverse volumes out)
    grad_div_volume: bool = True

    def __post_init__(self):
        g = self.grid
        self.a = g.face_vector(self.fr)
        self.l = g.edge_vector(self.fr)
        self.v = self.fr["v"].ravel().copy()
        self.Ct = curl_t(g)
        self.D = div(g)
        self.A = sp.diags(self.a)
        self.L = sp.diags(self.l)
        vinv = np.where(self.v > 0.0, 1.0 / np.where(self.v > 0.0, self.v, 1.0), 0.0)
        if not self.grad_div_volume:
            vinv = (self.v > 0.0).astype(float)
        self.Vinv = sp.diags(vinv)
        self.K = (self.Ct.T @ self.L @ self.Ct).tocsr()
        DA = (self.D @ self.A).tocsr()
        self.G = (DA.T @ self.Vinv @ DA).tocsr()
        self.M = (self.K + self.G - self.sigma * self.A).tocsr()
        self.S = (self.D @ self.A @ self.D.T).tocsr()
        self.act = np.flatnonzero(self.a > 0.0)
        self.cact = np.flatnonzero(self.v > 0.0)
        sel = self.act
        self.K_a = self.K[sel][:, sel].tocsr()
        self.G_a = self.G[sel][:, sel].tocsr()
        self.M_a = self.M[sel][:, sel].tocsr()
        self.a_a = self.a[sel]
        self.D_a = self.D[self.cact][:, sel].tocsr()   # cells x faces (active)
        self.S_a = self.S[self.cact][:, self.cact].tocsr()
        self.v_a = self.v[self.cact]

    def with_shift(self, sigma):
        return DMOperators(self.grid, self.fr, sigma, self.grad_div_volume)

    def full_face(self, x_active):
        """Scatter an active-face vector into the full face numbering."""
        out = np.zeros(self.grid.n_faces)
        out[self.act] = x_active
        return out


def build(fr, n, h, sigma=0.0, grad_div_volume=True) -> DMOperators:
    return DMOperators(YeeGrid(n, h), fr, sigma, grad_div_volume)


def apply_face_neglect(fr: dict, a_min: float) -> dict:
    """Face neglect of Sec. 3: faces with 0 < a < a_min are set to zero
    (their b is removed) and every edge of such a face gets l = 0.  A cell
    left without any open face holds no field; its volume is set to zero
    too (reading: otherwise its scalar unknown would be an isolated island
    of the projection's D A D^T)."""
    out = {k: v.copy() for k, v in fr.items()}
    nz, ny, nxp = fr["ax"].shape
    n = (nxp - 1, ny, nz)
    g = YeeGrid(n, 1.0)
    Ct = curl_t(g)
    a = g.face_vector(fr)
    drop = np.flatnonzero((a > 0.0) & (a < a_min))
    if drop.size == 0:
        return out
    edges = np.unique(Ct[:, drop].tocoo().row)
    a[drop] = 0.0
    l = g.edge_vector(fr)
    l[edges] = 0.0
    for s, arr in zip(("ax", "ay", "az"), g.split_faces(a)):
        out[s] = arr.copy()
    # cells with no open face among their six
    open_faces = abs(div(g)) @ (a > 0.0).astype(float)
    v = out["v"].ravel().copy()
    v[open_faces == 0.0] = 0.0
    out["v"] = v.reshape(fr["v"].shape)
    eoff = g.edge_off
    for ax, s in enumerate(("lx", "ly", "lz")):
        out[s] = l[eoff[ax]:eoff[ax + 1]].reshape(g.edge_shapes[ax]).copy()
    return out
