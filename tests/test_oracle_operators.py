"""Pins of the oracle's sparse operators (Secs. 2, 4 and 5).

Independent references: integer identities (D C = 0), the Kronecker-product
vector Laplacian of the PEC box (Dirichlet normal / Neumann tangential), the
closed-form box spectrum, and the identities stated in Sec. 5.1 and 5.2.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

from oracle import geometry as geo, operators as ops


def box_ops(n, sigma=0.0):
    h = 1.0 / n[0]
    fr = geo.fractions(geo.Box(), n, h)
    return ops.build(fr, n, h, sigma)


def random_fraction_ops(n, seed, sigma=0.0):
    """PEC box with every interior fraction drawn in [0.05, 1]: a generic
    cut-cell-like operator with no geometric structure."""
    h = 1.0 / n[0]
    fr = geo.fractions(geo.Box(), n, h)
    rng = np.random.default_rng(seed)
    for s in fr:
        fr[s] = np.where(fr[s] > 0, rng.uniform(0.05, 1.0, fr[s].shape), 0.0)
    return fr, ops.build(fr, n, h, sigma)


def test_div_curl_is_exactly_zero():
    """D C = 0 (Sec. 4.2, after eq. divB) as an integer stencil identity."""
    g = ops.YeeGrid((5, 4, 3), 1.0)
    DC = ops.div(g) @ ops.curl_t(g).T
    assert DC.nnz == 0 or abs(DC).max() == 0.0


def test_box_closed_form_spectrum_dense():
    """PEC unit cube, N = 4: nonzero eigenvalues of (K, A) are
    sum_a (2 sin(pi m_a / 2N) / h)^2 with at least two nonzero m_a,
    multiplicity 2 when all three are nonzero; the null space (gradients)
    has dimension N^3 - 1."""
    N = 4
    h = 1.0 / N
    op = box_ops((N, N, N))
    w = sl.eigh(op.K_a.toarray(), np.diag(op.a_a), eigvals_only=True)
    nz = np.sort(w[w > 1e-8 * w.max()])
    ref = []
    for m in itertools.product(range(N), repeat=3):
        if sum(x > 0 for x in m) < 2:
            continue
        lam = sum((2 * math.sin(math.pi * x / (2 * N)) / h) ** 2 for x in m)
        ref += [lam] * (2 if all(x > 0 for x in m) else 1)
    ref = np.sort(ref)
    assert op.act.size == 3 * (N - 1) * N * N
    assert len(nz) == len(ref) == 2 * (N - 1) ** 3 + 3 * (N - 1) ** 2
    assert np.sum(w <= 1e-8 * w.max()) == N ** 3 - 1
    assert np.max(abs(nz - ref) / ref) < 1e-13


def test_vacuum_box_decouples_into_scalar_laplacians():
    """In vacuum, K + G is block diagonal: each component sees the 7-point
    Laplacian, Dirichlet along its normal and Neumann across (Sec. 4.2,
    eq. discLaplB).  Reference built from 1-D second differences."""
    nx, ny, nz = 4, 3, 5
    h = 0.25
    fr = geo.fractions(geo.Box(), (nx, ny, nz), h)
    op = ops.build(fr, (nx, ny, nz), h, 0.0)
    KG = (op.K + op.G).tocsr()

    def dirichlet(m):  # interior nodes 1..m-1 of m cells
        return sp.diags([-1, 2, -1], [-1, 0, 1], shape=(m - 1, m - 1))

    def neumann(m):    # m cell-centred values, no flux through the walls
        T = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(m, m)).tolil()
        T[0, 0] = T[m - 1, m - 1] = 1
        return T.tocsr()

    g = op.grid
    sizes = (nx, ny, nz)
    for axis in range(3):
        # numbering of this component's interior faces in [k, j, i] C order
        mats = []
        for a in (2, 1, 0):  # k, j, i
            mats.append(dirichlet(sizes[a]) if a == axis else neumann(sizes[a]))
        eye = [sp.identity(m.shape[0]) for m in mats]
        lap = (sp.kron(sp.kron(mats[0], eye[1]), eye[2])
               + sp.kron(sp.kron(eye[0], mats[1]), eye[2])
               + sp.kron(sp.kron(eye[0], eye[1]), mats[2])) / h ** 2
        i, j, k = g.family(g.face_shapes[axis])
        idx = (i, j, k)
        inner = (idx[axis] > 0) & (idx[axis] < sizes[axis])
        fid = g.face(axis, i, j, k)[inner]
        block = KG[fid][:, fid].toarray()
        assert np.max(abs(block - lap.toarray())) < 1e-12
        others = np.setdiff1d(op.act, fid)
        assert abs(KG[fid][:, others]).max() == 0.0


def test_symmetry_and_semidefiniteness():
    fr, op = random_fraction_ops((4, 4, 4), seed=0, sigma=2.0)
    for Mx in (op.K, op.G, op.M, op.S):
        assert abs(Mx - Mx.T).max() <= 1e-13 * abs(Mx).max()
    for Mx in (op.K_a, op.G_a, op.S_a):
        w = np.linalg.eigvalsh(Mx.toarray())
        assert w.min() >= -1e-11 * w.max()


def test_spectrum_partition_random_fractions():
    """Sec. 5.1 (after eq. discLaplBDM): EM modes (lambda > 0 of (K, A)) are
    unchanged by the grad-div term, and the rest of spec(K + G, A) is the
    nonzero spectrum of (S, V) (gradient modes b = D^T psi)."""
    fr, op = random_fraction_ops((4, 4, 4), seed=0)
    a = op.a_a
    w_all = sl.eigh((op.K_a + op.G_a).toarray(), np.diag(a), eigvals_only=True)
    wk = sl.eigh(op.K_a.toarray(), np.diag(a), eigvals_only=True)
    ws = sl.eigh(op.S_a.toarray(), np.diag(op.v_a), eigvals_only=True)
    union = np.sort(np.concatenate([wk[wk > 1e-9 * wk.max()], ws[ws > 1e-9 * ws.max()]]))
    assert union.size == w_all.size
    assert np.max(abs(np.sort(w_all) - union) / union) < 1e-11


def test_spectrum_partition_sphere_6():
    n, h = (6, 6, 6), 1.0 / 6
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    op = ops.build(fr, n, h, 0.0)
    a = op.a_a
    w_all = sl.eigh((op.K_a + op.G_a).toarray(), np.diag(a), eigvals_only=True)
    wk = sl.eigh(op.K_a.toarray(), np.diag(a), eigvals_only=True)
    ws = sl.eigh(op.S_a.toarray(), np.diag(op.v_a), eigvals_only=True)
    union = np.sort(np.concatenate([wk[wk > 1e-9 * wk.max()], ws[ws > 1e-9 * ws.max()]]))
    assert union.size == w_all.size
    assert np.max(abs(np.sort(w_all) - union) / union) < 1e-10


def test_face_edge_duality():
    """Nonzero spectrum of A^-1/2 C L C^T A^-1/2 equals that of
    L^1/2 C^T A^-1 C L^1/2 (same singular values of A^-1/2 C L^1/2)."""
    fr, op = random_fraction_ops((3, 4, 3), seed=1)
    a = op.a
    l = op.l
    fa = a > 0
    el = l > 0
    Ct = op.Ct.toarray()
    B = (Ct[np.ix_(el, fa)] * np.sqrt(l[el])[:, None]) / np.sqrt(a[fa])[None, :]
    w1 = np.linalg.eigvalsh(B.T @ B)
    w2 = np.linalg.eigvalsh(B @ B.T)
    w1 = np.sort(w1[w1 > 1e-9 * w1.max()])
    w2 = np.sort(w2[w2 > 1e-9 * w2.max()])
    assert w1.size == w2.size
    assert np.max(abs(w1 - w2) / w1) < 1e-11


def test_face_neglect_removes_faces_and_their_edges():
    """Sec. 3: faces with a < a_min are dropped and every edge of a dropped
    face gets l = 0."""
    n, h = (8, 8, 8), 1.0 / 8
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    out = ops.apply_face_neglect(fr, 0.1)
    g = ops.YeeGrid(n, h)
    a0, a1 = g.face_vector(fr), g.face_vector(out)
    dropped = np.flatnonzero((a0 > 0) & (a0 < 0.1))
    assert dropped.size > 0
    assert np.all(a1[dropped] == 0.0)
    kept = np.flatnonzero(a0 >= 0.1)
    assert np.array_equal(a1[kept], a0[kept])
    Ct = ops.curl_t(g)
    edges = np.unique(Ct[:, dropped].tocoo().row)
    assert np.all(g.edge_vector(out)[edges] == 0.0)


def test_face_neglect_drops_cells_left_closed():
    """A cell all of whose six faces are neglected (here a box cell whose
    faces are made small by hand) gets v = 0; a cell keeping one open face
    keeps its volume."""
    n = (4, 4, 4)
    fr = geo.fractions(geo.Box(), n, 0.25)
    i, j, k = 1, 2, 1
    for s, idx in (("ax", [(k, j, i), (k, j, i + 1)]), ("ay", [(k, j, i), (k, j + 1, i)]),
                   ("az", [(k, j, i), (k + 1, j, i)])):
        for t in idx:
            fr[s][t] = 0.05
    out = ops.apply_face_neglect(fr, 0.1)
    assert out["v"][k, j, i] == 0.0
    assert np.count_nonzero(out["v"]) == 63
    fr["az"][k + 1, j, i] = 0.5          # one face stays open
    out = ops.apply_face_neglect(fr, 0.1)
    assert out["v"][k, j, i] == 1.0


def test_spectrum_partition_without_volumes_sphere_6():
    """The Sec. 6.1 variant without V^-1 (G0 = A D^T D A): the EM modes of
    (K, A) are still untouched, and the gradient branch becomes the nonzero
    spectrum of S itself (V replaced by the identity), so the variant moves
    only the gradient modes -- which is why it can change the solver's
    convergence and not the eigenpairs."""
    n, h = (6, 6, 6), 1.0 / 6
    fr = geo.fractions(geo.sphere((0.5, 0.5, 0.5), 0.45), n, h)
    op = ops.build(fr, n, h, 0.0, grad_div_volume=False)
    a = op.a_a
    w_all = sl.eigh((op.K_a + op.G_a).toarray(), np.diag(a), eigvals_only=True)
    wk = sl.eigh(op.K_a.toarray(), np.diag(a), eigvals_only=True)
    ws = sl.eigvalsh(op.S_a.toarray())
    union = np.sort(np.concatenate([wk[wk > 1e-9 * wk.max()], ws[ws > 1e-9 * ws.max()]]))
    assert union.size == w_all.size
    assert np.max(abs(np.sort(w_all) - union) / union) < 1e-10
    # and it differs from the method's G exactly where cut cells have v < 1
    full = ops.build(fr, n, h, 0.0)
    assert abs(full.G_a - op.G_a).max() > 0.1 * abs(full.G_a).max()
